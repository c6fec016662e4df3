"""Benchmark: HISQ even/odd Dslash GB/s against the HBM roofline, and CG time
to |r|/|b| < 1e-10, plain FP64 CG vs the mixed-precision form.

One timed step = one FP32 single-parity Dslash over the whole 96^3 x 24
lattice (one GPU's share of a large-volume HISQ lattice), 1 RHS, inputs
resident in HBM.  Around it the run also measures the FP64 / FP16S /
multi-RHS Dslash variants, the 96^3 x 24 time to solution (plain FP64 CG
against the chosen form: 4 RHS batched, mixed FP32/FP64), CG solves at
32^3 x 8 (plain FP64 vs mixed FP32 and FP16S with reliable updates),
batched, multi-shift and rational solves at 48^3 x 12, the network
preconditioner, and - the CPU-baseline leg, the only one that runs the FP64
oracle - the oracle's own Dslash on the host cores, whose output must match
the timed launch's, and the oracle's true residual of every solution.

Every workload's gauge field is generated before the GPU is first used.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
Prints ONE JSON line on stdout; progress goes to stderr.
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

HBM_PEAK_GBS = 8000.0
FLOP_PER_SITE = 1146
METRIC = "Dslash GB/s (% HBM peak); CG time to |r|/|b|<1e-10, plain vs chosen form"


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def cb_gather(dims, vec_full, parity):
    """[V,3] full-lattice vector -> [3, Vh] values of one parity (checkerboard order)."""
    from paper_2111_10354_amd import layout
    s = layout.parity_sites(dims, parity)
    return layout.to_planes(vec_full, s), s


def encode(cb, prec):
    from paper_2111_10354_amd import layout
    return layout.encode(cb, prec)


def counter_traffic(dims, compressed, shape):
    """HBM bytes per launch of the headline kernel from the committed rocprofv3
    counter summary, or None if the kernel sources, the link layout or the
    launch shape (RHS tile, block, tile order) changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"dslash_fp32_{'x'.join(map(str, dims))}.traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    csrc = os.path.join(ROOT, "paper_2111_10354_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, n), "rb").read() for n in ("dslash.hip", "hisq_internal.h", "pack.hip"))
    if hashlib.sha256(src).hexdigest() != rec.get("kernel_sources_sha256"):
        return None
    if bool(rec.get("long_links_compressed", False)) != bool(compressed):
        return None
    if rec.get("launch_shape") != [int(v) for v in shape]:
        return None
    return rec["traffic_bytes_per_launch"] / 1e9  # GB, like `achieved`


def time_launches(fn, steps, warmup):
    """Average time of fn() (launches on the current stream) from HIP events."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps  # ms


def generate_fields(which, dims_c5):
    """Every workload's links, generated up front (before the GPU is used): the
    worker pool forks only from a process without GPU state."""
    import synth
    out = {}
    for name in which:
        c = synth.CONFIGS[name]
        dims = dims_c5 if name == "c5" else c["dims"]
        t0 = time.time()
        if name == "c5":  # the unfolded thin links too: the smearing leg starts from them
            F, L, U = synth.fields.hisq_links_and_thin(dims, synth.CFG_IDS[name], c["eps"])
            out[name], out["c5_thin"] = (F, L), U
        else:
            out[name] = synth.hisq_links(dims, synth.CFG_IDS[name], c["eps"], want_thin=(name == "c4"))
        log(f"fields {name} {dims} (eps={c['eps']}): {time.time() - t0:.1f}s")
    return out


def run_smeared(hisq, torch, tune, dims, U, nrhs):
    """HISQ smearing of the 96^3 x 24 thin links on the GPU, and the FP32 Dslash
    on the smeared links (Naik links stored as two rows and a complex factor)."""
    import synth
    vh = synth.volume(dims) // 2
    t = torch.from_numpy(U).cuda()
    fat, lng = torch.empty_like(t), torch.empty_like(t)
    hisq.smear_links(dims, t, fat, lng)  # first call: code objects loaded
    torch.cuda.synchronize()
    t1 = time.time()
    hisq.smear_links(dims, t, fat, lng)
    torch.cuda.synchronize()
    t_smear = time.time() - t1
    del t
    g = hisq.Gauge(dims, fat, lng, ("fp32",))
    del fat, lng
    torch.cuda.empty_cache()
    out = {"workload": f"{'x'.join(map(str, dims))}: HISQ smearing (fat7, U(3) projection, fat7 + Lepage, Naik) "
                       "of the thin links in FP64, then the FP32 Dslash on the smeared links",
           "smear_seconds": round(t_smear, 4), "naik_compression_mode": g.comp_mode}
    real = 4
    link = real * (8 * 18 + 8 * 12 + 8 * 2) if g.comp_mode == 2 else real * 16 * 18
    for n in (1, nrhs):
        hisq.autotune(g, "fp32", n, tune)
        nb = hisq.spinor_bytes("fp32", vh) * n
        i = torch.randn(nb // 4, device="cuda").view(torch.uint8)
        o = torch.empty_like(i)
        ms = time_launches(lambda: hisq.dslash_multi_rhs(g, 0, "fp32", n, i, o), 20, 5)
        gbs = vh * (link + 2 * 24 * n) / (ms * 1e-3) / 1e9
        out[f"fp32_x{n}rhs"] = {"ms": round(ms, 4), "gbs": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                                "shape": list(hisq.dslash_shape(g, "fp32", n, 0))}
        log(f"smeared links: FP32 Dslash {n} RHS {ms:.3f} ms, {gbs:.0f} GB/s")
        del i, o
    log(f"smearing {dims}: {t_smear:.3f} s")
    g.close()
    return out


def oracle_residuals(dims, F, L, mass, items):
    """The oracle's FP64 true residual |b - (A + sigma) x| / |b| of every
    (name, b, x, sigma) solution (full-lattice host vectors)."""
    import oracle
    out = {}
    for name, b, x, sigma in items:
        out[name] = oracle.true_residual(dims, F, L, mass, b, x, sigma=sigma)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    # 200 launches (~0.4 s) bring the GPU to its steady state; 10 left the
    # headline 2-4 % slow on some boxes
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--dims", type=str, default="96,96,96,24")
    ap.add_argument("--quick", action="store_true", help="skip the solves and the CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--no-c5", action="store_true", help="skip the 96^3x24 time to solution")
    ap.add_argument("--no-nn", action="store_true", help="skip the preconditioner network training and FCG")
    ap.add_argument("--c5-solve", action="store_true",
                    help="only the 96^3x24, m=0.002, 4-RHS solve: chosen form against plain FP64 CG (minutes)")
    ap.add_argument("--c5-fp16s", action="store_true",
                    help="with --c5-solve: also the FP16S-sloppy batched solve (~10 minutes at this mass)")
    ap.add_argument("--only-fp32", action="store_true", help="time only the headline kernel")
    ap.add_argument("--tune-cache", type=str, default=os.path.join(ROOT, "paper_2111_10354_amd", "tuning",
                                                                  "gfx950.jsonl"),
                    help="autotuner cache (JSON lines); shapes found there are used without timing")
    ap.add_argument("--no-sweep", action="store_true", help="skip the 48^3x12 multi-RHS sweep")
    ap.add_argument("--no-c3", action="store_true", help="skip the 48^3x12 batched and multi-shift solves")
    ap.add_argument("--c2-dslash", action="store_true",
                    help="only the 32^3x8 single-RHS Dslash in FP64, FP32 and FP16S (for counter runs)")
    ap.add_argument("--c3-solvers", action="store_true",
                    help="only the 48^3x12 solves (plain, mixed, 16-RHS batched, 12-shift, A^(-1/2))")
    ap.add_argument("--fields-cache", type=str, default=None,
                    help="directory to save / reuse the generated 96^3x24 link fields (profiling re-runs)")
    ap.add_argument("--mrhs", type=int, default=0,
                    help="only the N-RHS FP32 Dslash on the --dims lattice (long links compressed unless --full-links), "
                         "for profiling: --shape forces a launch shape")
    ap.add_argument("--shape", type=str, default=None, help="with --mrhs: tile,block,order")
    ap.add_argument("--full-links", action="store_true", help="with --mrhs: store every link whole")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 4 GiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = 4 << 30
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        ms = time_launches(lambda: dst.copy_(src), 5, 1)
        log(f"copy of {n >> 20} MiB: {ms:.3f} ms, {2 * n / (ms * 1e-3) / 1e9:.0f} GB/s (read+write)")
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "ms": ms,
                          "gbs_read_plus_write": 2 * n / (ms * 1e-3) / 1e9}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the lattice would be split by domain decomposition with halo exchange; not built)",
              file=sys.stderr)
        sys.exit(2)

    import synth  # input generator only
    # minutes-long solves (the 96^3x24 ones): the library prints its progress
    # every 2000 iterations to stderr, so a long run is never silent
    os.environ.setdefault("HISQ_SOLVER_TRACE", "1")
    tune = args.tune_cache if args.tune_cache and os.path.isdir(os.path.dirname(args.tune_cache)) else None
    dims = tuple(int(v) for v in args.dims.split(","))
    if args.c3_solvers:
        fl = generate_fields(("c3",), dims)
        import torch
        from paper_2111_10354_amd import hisq
        out, _ = run_c3_solvers(hisq, torch, tune, fl["c3"], extended=True)
        print(json.dumps(out), flush=True)
        return
    if args.c2_dslash:
        fl = generate_fields(("c2",), dims)
        import torch
        from paper_2111_10354_amd import hisq
        print(json.dumps(run_c2_dslash(hisq, torch, tune, fl["c2"], args.steps, min(args.warmup, 50))), flush=True)
        return
    if args.mrhs:
        run_mrhs_only(args, dims, tune)
        return
    if args.c5_solve:
        fl = generate_fields(("c5",), dims)
        import torch
        from paper_2111_10354_amd import hisq
        out, _ = run_c5_solve(hisq, torch, tune, dims, *fl["c5"], with_fp16s=args.c5_fp16s)
        print(json.dumps(out), flush=True)
        return

    V = synth.volume(dims)
    vh = V // 2
    cfg = synth.CONFIGS["c5"]
    full = not (args.quick or args.only_fp32)
    want = ["c5"]
    if full and not args.no_sweep or full and not (args.no_cg or args.no_c3):
        want.append("c3")
    if full and not args.no_cg:
        want.append("c2")
    if full and not args.no_nn:
        want.append("c4")
    cache = None
    if args.fields_cache:
        tag = f"hisq_{'x'.join(map(str, dims))}_c5_eps{cfg['eps']}"
        cache = (os.path.join(args.fields_cache, tag + "_fat.npy"), os.path.join(args.fields_cache, tag + "_long.npy"))
    if cache and all(os.path.exists(p) for p in cache):
        log(f"loading cached fields {cache[0]}")
        fields = {"c5": (np.load(cache[0]), np.load(cache[1]))}
        fields.update(generate_fields([w for w in want if w != "c5"], dims))
    else:
        fields = generate_fields(want, dims)
        if cache:
            os.makedirs(args.fields_cache, exist_ok=True)
            np.save(cache[0], fields["c5"][0])
            np.save(cache[1], fields["c5"][1])
    F, L = fields["c5"]
    chi = synth.gaussian_source(dims, synth.CFG_IDS["c5"], 1, parity=1)[0]

    import torch
    from paper_2111_10354_amd import hisq

    # every precision is packed even when only FP32 is timed, so that the
    # headline kernel's buffers sit where they sit in the default run
    precs = ("fp64", "fp32", "fp16s")

    def make_gauge(full_links):
        fd, ld = torch.from_numpy(F).cuda(), torch.from_numpy(L).cuda()
        gx = hisq.Gauge(dims, fd, ld, precs, full_links=full_links)
        torch.cuda.synchronize()
        del fd, ld
        torch.cuda.empty_cache()
        t1 = time.time()
        for p in precs:
            for n in (1, cfg["nrhs"]):
                hisq.autotune(gx, p, n, tune)
        log(f"gauge ({'links whole' if full_links else 'long links compressed' if gx.compressed else 'links whole'}): "
            f"{gx.device_bytes() / 2**30:.1f} GiB; autotune ({'cache ' + tune if tune else 'no cache'}) "
            f"{time.time() - t1:.1f}s; FP32 1-RHS shape {hisq.dslash_shape(gx, 'fp32', 1, 0)}")
        return gx

    # the headline kernel reads every link whole: its GB/s measures bandwidth
    # efficiency on the full 1200 B/site; the compressed layout is timed below
    g = make_gauge(True)

    cb, odd_sites = cb_gather(dims, chi, 1)
    bufs = {}
    for p in precs:
        inp = torch.from_numpy(encode(cb, p)).cuda()
        out = torch.empty(hisq.spinor_bytes(p, vh), dtype=torch.uint8, device="cuda")
        bufs[p] = (inp, out)

    def algo_bytes(p, nrhs=1, comp=0):
        real = {"fp64": 8, "fp32": 4, "fp16s": 2}[p]
        if p == "fp64" or not comp:
            link = real * 16 * 18
        elif comp == 1:  # two rows + a sign word per site
            link = real * (8 * 18 + 8 * 12) + 4
        else:            # two rows + a complex factor per long link
            link = real * (8 * 18 + 8 * 12 + 8 * 2)
        spin = {"fp64": 48, "fp32": 24, "fp16s": 16}[p]
        return vh * (link + nrhs * 2 * spin)

    # ---- headline: FP32 single-RHS single-parity Dslash
    inp, out = bufs["fp32"]
    ms = time_launches(lambda: hisq.dslash_eo(g, 0, "fp32", inp, out), args.steps, args.warmup)
    gbs = algo_bytes("fp32") / (ms * 1e-3) / 1e9
    log(f"FP32 Dslash: {ms:.3f} ms/launch, {gbs:.0f} GB/s algorithmic ({100 * gbs / HBM_PEAK_GBS:.1f}% of 8 TB/s)")

    # the timed launch's output, compared with the oracle in the CPU-baseline leg
    torch.cuda.synchronize()
    from paper_2111_10354_amd import layout
    got_fp32 = layout.decode(out.cpu().numpy(), vh, "fp32")

    variants = {"fp32": {"ms": ms, "gbs": gbs}}
    shape = hisq.dslash_shape(g, "fp32", 1, 0)

    def time_variants(gx, comp, suffix, skip_fp32):
        for p in ("fp64", "fp32", "fp16s"):
            if (p == "fp32" and skip_fp32) or (p == "fp64" and comp):
                continue  # the FP64 copy always keeps its links whole
            i2, o2 = bufs[p]
            m2 = time_launches(lambda: hisq.dslash_eo(gx, 0, p, i2, o2), max(10, args.steps // 2), 3)
            variants[p + suffix] = {"ms": m2, "gbs": algo_bytes(p, comp=comp) / (m2 * 1e-3) / 1e9}
            log(f"{p}{suffix} Dslash: {m2:.3f} ms, {variants[p + suffix]['gbs']:.0f} GB/s")
        # 4 RHS (the workload's batch) through the multi-RHS kernel
        n = cfg["nrhs"]
        srcs = synth.gaussian_source(dims, synth.CFG_IDS["c5"], n, parity=1, index0=1)
        for p in ("fp32", "fp16s"):
            raw = np.concatenate([encode(cb_gather(dims, s_, 1)[0], p) for s_ in srcs])
            i4 = torch.from_numpy(raw).cuda()
            o4 = torch.empty(hisq.spinor_bytes(p, vh) * n, dtype=torch.uint8, device="cuda")
            m4 = time_launches(lambda: hisq.dslash_multi_rhs(gx, 0, p, n, i4, o4), max(10, args.steps // 2), 3)
            key = f"{p}_x{n}rhs{suffix}"
            variants[key] = {"ms": m4, "gbs": algo_bytes(p, n, comp=comp) / (m4 * 1e-3) / 1e9, "ms_per_rhs": m4 / n,
                             "shape": list(hisq.dslash_shape(gx, p, n, 0))}
            log(f"{key} Dslash: {m4:.3f} ms ({m4 / n:.3f} ms/RHS), {variants[key]['gbs']:.0f} GB/s")
            del i4, o4

    c5 = None
    solutions = {}
    if not args.only_fp32:
        time_variants(g, 0, "", True)
        # long links as two rows + determinant sign (the layout the solvers use)
        g.close()
        torch.cuda.empty_cache()
        g = make_gauge(False)
        if g.compressed:
            time_variants(g, g.comp_mode, "_compressed", False)
        if not (args.quick or args.no_cg or args.no_c5):
            c5, solutions["c5"] = run_c5_solve(hisq, torch, tune, dims, F, L, gauge=g)
    for k, v in variants.items():
        v["gflops"] = FLOP_PER_SITE * vh * (4 if "x4" in k else 1) / (v["ms"] * 1e-3) / 1e9
        v["frac_hbm_peak"] = v["gbs"] / HBM_PEAK_GBS
    del bufs
    g.close()
    torch.cuda.empty_cache()
    smeared = None
    if full and "c5_thin" in fields:
        smeared = run_smeared(hisq, torch, tune, dims, fields.pop("c5_thin"), cfg["nrhs"])
    sweep = None
    if full and not args.no_sweep:
        sweep = run_mrhs_sweep(hisq, torch, tune, fields["c3"])

    # ---- CG time to solution on the 32^3 x 8 workload, and its Dslash per precision
    cg = None
    if full and not args.no_cg:
        cg, solutions["c2"] = run_cg(hisq, torch, fields["c2"])
        cg["dslash_single_rhs"] = run_c2_dslash(hisq, torch, tune, fields["c2"], 200, 50)

    # ---- batched and multi-shift solves on the 48^3 x 12 workload
    c3 = None
    if full and not (args.no_cg or args.no_c3):
        c3, solutions["c3"] = run_c3_solvers(hisq, torch, tune, fields["c3"])

    # ---- network preconditioner on the 32^3 x 8, m = 0.005 workload
    nnres = None
    if full and not args.no_nn:
        nnres, solutions["c4"] = run_nn(hisq, torch, fields["c4"])

    # ---- CPU baseline: the FP64 oracle's Dslash on this lattice, host cores;
    # the timed launch's output and every solution checked by the oracle
    cpu = None
    perr = None
    residuals = None
    if not (args.quick or args.no_cpu):
        import oracle  # test infrastructure: the CPU baseline and the checks of the GPU results
        nthr = oracle.num_threads()
        log(f"oracle Dslash on the host ({nthr} threads)")
        reps, t_tot = 0, 0.0
        while t_tot < 2.0 and reps < 4:
            t1 = time.time()
            want = oracle.dslash(dims, F, L, chi, 0)
            t_tot += time.time() - t1
            reps += 1
        # every output site of the timed FP32 launch against the oracle (whose
        # input is not rounded to FP32: the difference includes that rounding)
        want_cb = cb_gather(dims, want, 0)[0]
        perr = float(np.linalg.norm(got_fp32 - want_cb) / np.linalg.norm(want_cb))
        log(f"FP32 Dslash vs oracle over all {vh} output sites: rel L2 {perr:.2e}")
        del want, want_cb
        if not perr <= 1e-6:
            log(f"FAIL: the timed FP32 Dslash differs from the oracle by {perr:.2e} > 1e-6")
            sys.exit(1)
        t_one = t_tot / reps
        cpu = {"value": algo_bytes("fp64") / t_one / 1e9, "unit": "GB/s", "cores": nthr, "kind": "oracle",
               "sample": f"{reps} full single-parity FP64 Dslash applications on the same {dims} lattice "
                         f"({t_one:.2f} s each); GB/s counts the FP64 algorithmic bytes (2400 B/site)"}
        log(f"oracle: {t_one:.2f} s per Dslash = {cpu['value']:.2f} GB/s")
        if "c2" in fields:
            # the oracle's plain FP64 CG on the 32^3 x 8 workload: 200 iterations
            # timed, the time to solution extrapolated to the GPU's iteration count
            c2 = synth.CONFIGS["c2"]
            F2, L2 = fields["c2"]
            b2 = synth.gaussian_source(c2["dims"], synth.CFG_IDS["c2"], 1, parity=0)[0]
            t1 = time.time()
            _, _, it2, _ = oracle.cg(c2["dims"], F2, L2, c2["mass"], b2, tol=1e-10, max_iter=200)
            per_it = (time.time() - t1) / max(it2, 1)
            cpu["cg_32x32x32x8"] = {"seconds_per_iteration": per_it, "iterations_timed": it2,
                                    "note": "plain FP64 CG of the oracle; time to solution = this x the GPU's "
                                            "plain-CG iteration count (extrapolated)"}
            if cg is not None:
                cpu["cg_32x32x32x8"]["extrapolated_seconds_to_solution"] = per_it * cg["plain_fp64"]["iterations"]
            log(f"oracle CG 32^3x8: {1e3 * per_it:.1f} ms per iteration ({it2} timed)")
        # the oracle's whole plain CG on the 8^4 workload (seconds), one A
        # application on the benchmark lattice, and per-iteration time on 48^3 x 12
        c1 = synth.CONFIGS["c1"]
        F1, L1 = synth.hisq_links(c1["dims"], synth.CFG_IDS["c1"], c1["eps"])
        b1 = synth.gaussian_source(c1["dims"], synth.CFG_IDS["c1"], 1, parity=0)[0]
        t1 = time.time()
        _, st1, it1, tr1 = oracle.cg(c1["dims"], F1, L1, c1["mass"], b1, tol=1e-10)
        cpu["cg_8x8x8x8"] = {"seconds_to_solution": time.time() - t1, "iterations": it1, "status": st1,
                             "true_residual": tr1}
        log(f"oracle CG 8^4: {cpu['cg_8x8x8x8']['seconds_to_solution']:.3f} s, {it1} iterations")
        ev = synth.gaussian_source(dims, synth.CFG_IDS["c5"], 1, parity=0)[0]
        t1 = time.time()
        oracle.normal_op(dims, F, L, cfg["mass"], ev)
        cpu["normal_op_seconds"] = time.time() - t1
        del ev
        log(f"oracle A application on {dims}: {cpu['normal_op_seconds']:.2f} s")
        if "c3" in fields and c3 is not None:
            c3c = synth.CONFIGS["c3"]
            F3, L3 = fields["c3"]
            b3 = synth.gaussian_source(c3c["dims"], synth.CFG_IDS["c3"], 1, parity=0)[0]
            t1 = time.time()
            _, _, it3, _ = oracle.cg(c3c["dims"], F3, L3, c3c["mass"], b3, tol=1e-10, max_iter=30)
            per3 = (time.time() - t1) / max(it3, 1)
            cpu["cg_48x48x48x12"] = {
                "seconds_per_iteration": per3, "iterations_timed": it3,
                "extrapolated_seconds_to_solution": per3 * c3["plain_fp64_1rhs"]["iterations_max"],
                "note": "plain FP64 CG of the oracle; x the GPU's plain-CG iteration count (extrapolated)"}
            log(f"oracle CG 48^3x12: {1e3 * per3:.1f} ms per iteration ({it3} timed)")
        # the oracle's true residual of every solution of the run
        residuals = {}
        t1 = time.time()
        for name, (cdims, mass, items) in solutions.items():
            Fx, Lx = fields[name][0], fields[name][1]
            residuals[name] = oracle_residuals(cdims, Fx, Lx, mass, items)
        worst = max((v for r in residuals.values() for v in r.values()), default=0.0)
        residuals["worst"] = worst
        log(f"oracle true residuals of {sum(len(r) for k, r in residuals.items() if k != 'worst')} solutions "
            f"({time.time() - t1:.1f}s): worst {worst:.3e}")
    del F, L

    result = {
        "metric": METRIC,
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"HISQ single-parity Dslash, {'x'.join(map(str, dims))} lattice, FP32 links "
                               f"(all stored whole) and spinors, 1 RHS, seeded links (eps={cfg['eps']})",
                   "long_links_compressed": False,
                   "dims": list(dims), "sites_per_parity": vh, "bytes_per_step": algo_bytes("fp32"),
                   "flop_per_site": FLOP_PER_SITE},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": counter_traffic(dims, False, shape),
                     "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"},
        "cpu_baseline": cpu,
        "parity_rel_l2_vs_oracle": perr,
        "oracle_true_residuals": residuals,
        "time_to_solution_96x96x96x24": c5,
        "smeared_links_96x96x96x24": smeared,
        "variants": variants,
        "cg": cg,
        "c3_solvers": c3,
        "nn_fcg": nnres,
    }
    result["config"]["launch_shape"] = {"rhs_tile": shape[0], "block": shape[1], "tile_order": shape[2]}
    result["mrhs_sweep"] = sweep
    print(json.dumps(result), flush=True)
    if residuals and not residuals["worst"] <= 1e-10:
        log(f"FAIL: a reported solution's oracle true residual is {residuals['worst']:.3e} > 1e-10")
        sys.exit(1)


def run_mrhs_sweep(hisq, torch, tune, fields):
    """Multi-RHS Dslash on 48^3 x 12 (FP32 and FP16S): time per launch and per RHS
    for N = 1, 2, 4, 8, 16 with autotuned shapes."""
    import synth
    c = synth.CONFIGS["c3"]
    dims = c["dims"]
    vh = synth.volume(dims) // 2
    F, L = fields
    g = hisq.Gauge(dims, torch.from_numpy(F).cuda(), torch.from_numpy(L).cuda(), ("fp32", "fp16s"))
    srcs = synth.gaussian_source(dims, synth.CFG_IDS["c3"], 16, parity=1)
    out = {"workload": f"{'x'.join(map(str, dims))} single-parity Dslash, N right-hand sides",
           "long_links_compressed": g.compressed, "fp32": {}, "fp16s": {}}
    for p in ("fp32", "fp16s"):
        raw = np.concatenate([encode(cb_gather(dims, s, 1)[0], p) for s in srcs])
        i16 = torch.from_numpy(raw).cuda()
        o16 = torch.empty_like(i16)
        real = {"fp32": 4, "fp16s": 2}[p]
        link = real * (8 * 18 + 8 * 12) + 4 if g.compressed else real * 16 * 18
        spin = {"fp32": 24, "fp16s": 16}[p]
        for n in (1, 2, 4, 8, 16):
            hisq.autotune(g, p, n, tune)
            nb = hisq.spinor_bytes(p, vh) * n
            ms = time_launches(lambda: hisq.dslash_multi_rhs(g, 0, p, n, i16[:nb], o16[:nb]), 20, 3)
            gbs = vh * (link + 2 * spin * n) / (ms * 1e-3) / 1e9
            out[p][str(n)] = {"ms": round(ms, 4), "ms_per_rhs": round(ms / n, 4), "gbs": round(gbs, 1),
                              "gflops": round(1146 * vh * n / (ms * 1e-3) / 1e9, 1),
                              "shape": list(hisq.dslash_shape(g, p, n, 0))}
            log(f"sweep {p} N={n}: {ms:.3f} ms ({ms / n:.3f} ms/RHS), {gbs:.0f} GB/s")
    g.close()
    return out


def _host_solution(dims, xdev, vh, index=0):
    """Full-lattice host vector of RHS `index` of an FP64 even-site solution stack."""
    from paper_2111_10354_amd import layout
    import synth
    sb = 48 * vh
    raw = xdev[index * sb:(index + 1) * sb].cpu().numpy()
    full = np.zeros((synth.volume(dims), 3), np.complex128)
    full[layout.parity_sites(dims, 0)] = layout.decode(raw, vh, "fp64").T
    return full


def run_cg(hisq, torch, fields):
    import synth
    c = synth.CONFIGS["c2"]
    dims, mass = c["dims"], c["mass"]
    vh = synth.volume(dims) // 2
    F, L = fields
    g = hisq.Gauge(dims, torch.from_numpy(F).cuda(), torch.from_numpy(L).cuda(), ("fp64", "fp32", "fp16s"))
    b = synth.gaussian_source(dims, synth.CFG_IDS["c2"], 1, parity=0)[0]
    bcb, _ = cb_gather(dims, b, 0)
    bd = torch.from_numpy(encode(bcb, "fp64")).cuda()
    out = {"workload": f"{'x'.join(map(str, dims))}, m={mass}, 1 Gaussian RHS, tol 1e-10 (true residual)"}
    items = []
    for name, sloppy in (("plain_fp64", "fp64"), ("mixed_fp32", "fp32"), ("mixed_fp16s", "fp16s")):
        prm = hisq.solver_params(sloppy_prec=sloppy, graph_chunk=25)
        x = torch.zeros_like(bd)
        hisq.cg_solve(g, mass, 1, bd, x, hisq.solver_params(sloppy_prec=sloppy, graph_chunk=25, max_iter=50))
        x.zero_()
        torch.cuda.synchronize()
        t1 = time.time()
        rc, st = hisq.cg_solve(g, mass, 1, bd, x, prm)
        wall = time.time() - t1
        out[name] = {"status": rc, "seconds": round(wall, 4), "iterations": st[0]["iterations"],
                     "reliable_updates": st[0]["reliable_updates"],
                     "true_residual": st[0]["true_residual"]}
        items.append((name, b, _host_solution(dims, x, vh), 0.0))
        log(f"CG {name}: {wall:.3f} s, {st[0]['iterations']} it, true res {st[0]['true_residual']:.2e}")
    best = min(("mixed_fp32", "mixed_fp16s"), key=lambda k: out[k]["seconds"] if out[k]["status"] == 0 else 1e30)
    out["chosen"] = best
    out["speedup_chosen_vs_plain"] = round(out["plain_fp64"]["seconds"] / out[best]["seconds"], 3)
    g.close()
    return out, (dims, mass, items)


def link_bytes_per_site(prec, comp):
    """Algorithmic link bytes of one output site: 16 links, the long ones as
    two rows plus a sign word (comp 1) or a complex factor (comp 2)."""
    real = {"fp64": 8, "fp32": 4, "fp16s": 2}[prec]
    if prec == "fp64" or not comp:
        return real * 16 * 18
    return real * (8 * 18 + 8 * 12) + (4 if comp == 1 else real * 16)


def run_c2_dslash(hisq, torch, tune, fields, steps, warmup):
    """Single-RHS single-parity Dslash on 32^3 x 8 in FP64, FP32 and FP16S
    (long links compressed as the solvers use them; FP64 links whole), timed
    with HIP events.  The FP32 links (120 MiB) fit in the 256 MB Infinity
    Cache, so back-to-back launches can read them from there: the counter
    summary in profiles/ gives the bytes that left the L2s."""
    import synth
    c = synth.CONFIGS["c2"]
    dims = c["dims"]
    vh = synth.volume(dims) // 2
    F, L = fields
    g = hisq.Gauge(dims, torch.from_numpy(F).cuda(), torch.from_numpy(L).cuda(), ("fp64", "fp32", "fp16s"))
    chi = synth.gaussian_source(dims, synth.CFG_IDS["c2"], 1, parity=1)[0]
    ccb, _ = cb_gather(dims, chi, 1)
    res = {"workload": f"{'x'.join(map(str, dims))} single-parity Dslash, 1 RHS",
           "long_links": ["whole", "sign", "kappa"][g.comp_mode]}
    for p in ("fp64", "fp32", "fp16s"):
        hisq.autotune(g, p, 1, tune)
        i1 = torch.from_numpy(encode(ccb, p)).cuda()
        o1 = torch.empty(hisq.spinor_bytes(p, vh), dtype=torch.uint8, device="cuda")
        ms = time_launches(lambda: hisq.dslash_eo(g, 0, p, i1, o1), steps, warmup)
        spin = hisq.spinor_bytes(p, vh) // vh
        gbs = vh * (link_bytes_per_site(p, g.comp_mode) + 2 * spin) / (ms * 1e-3) / 1e9
        res[p] = {"ms": round(ms, 5), "gbs": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                  "shape": list(hisq.dslash_shape(g, p, 1, 0))}
        log(f"C2 {p} Dslash: {ms:.4f} ms, {gbs:.0f} GB/s algorithmic, shape {res[p]['shape']}")
        del i1, o1
    g.close()
    return res


def run_mrhs_only(args, dims, tune):
    """One N-RHS FP32 Dslash shape on the benchmark lattice, timed with HIP events
    (for counter runs: the launches of the timed loop are the last ones)."""
    import synth
    import torch
    from paper_2111_10354_amd import hisq
    n = args.mrhs
    cache = None
    if args.fields_cache:
        cfg = synth.CONFIGS["c5"]
        tag = f"hisq_{'x'.join(map(str, dims))}_c5_eps{cfg['eps']}"
        cache = (os.path.join(args.fields_cache, tag + "_fat.npy"), os.path.join(args.fields_cache, tag + "_long.npy"))
    if cache and all(os.path.exists(p) for p in cache):
        F, L = np.load(cache[0]), np.load(cache[1])
    else:
        F, L = generate_fields(["c5"], dims)["c5"]
        if cache:
            os.makedirs(args.fields_cache, exist_ok=True)
            np.save(cache[0], F)
            np.save(cache[1], L)
    g = hisq.Gauge(dims, torch.from_numpy(F).cuda(), torch.from_numpy(L).cuda(), ("fp32",),
                   full_links=args.full_links)
    del F, L
    table = tune
    if args.shape:
        t, b, o = (int(v) for v in args.shape.split(","))
        table = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"hisq_shape_{os.getpid()}.jsonl")
        probe = table + ".probe"
        hisq.autotune(g, "fp32", n, probe)  # writes this handle's keys
        keys = [json.loads(line)["key"] for line in open(probe)]
        with open(table, "w") as f:
            for k in keys:
                if f"|n{n}|e0" in k:
                    f.write(json.dumps({"key": k, "tile": t, "block": b, "order": o, "ms": 0.0}) + "\n")
        os.remove(probe)
    hisq.autotune(g, "fp32", n, table)
    shape = tuple(hisq.dslash_shape(g, "fp32", n, 0))
    if args.shape:
        os.remove(table)
        assert shape == (t, b, o), (shape, args.shape)
    vh = synth.volume(dims) // 2
    nb = hisq.spinor_bytes("fp32", vh)
    inp = torch.randn(n * nb // 4, device="cuda").view(torch.uint8)
    out = torch.empty(n * nb, dtype=torch.uint8, device="cuda")
    ms = time_launches(lambda: hisq.dslash_multi_rhs(g, 0, "fp32", n, inp, out), args.steps, args.warmup)
    comp = g.comp_mode
    link = 4 * 16 * 18 if comp == 0 else 4 * (8 * 18 + 8 * 12) + 4 if comp == 1 else 4 * (8 * 18 + 8 * 12 + 16)
    gbs = vh * (link + n * 48) / (ms * 1e-3) / 1e9
    log(f"{n}-RHS FP32 Dslash, shape {shape}: {ms:.4f} ms, {gbs:.0f} GB/s algorithmic")
    print(json.dumps({"workload": f"{'x'.join(map(str, dims))} single-parity FP32 Dslash, {n} RHS",
                      "long_links": ["whole", "sign", "kappa"][comp], "shape": shape, "ms": ms, "gbs": gbs,
                      "steps": args.steps, "warmup": args.warmup}), flush=True)
    g.close()


def run_c3_solvers(hisq, torch, tune, fields, extended=False):
    """48^3 x 12, m = 0.005: one RHS by plain FP64 CG and by mixed FP32 CG, all
    16 RHS batched through the multi-RHS Dslash (mixed FP32, FP64 reliable
    updates), the 12-shift ladder sigma_k = 10^(-4 + 4k/11) by multi-shift CG,
    and the two-flavour pseudofermion heat bath phi = A^(1/4) eta (16 Remez
    poles) and action phi^+ A^(-1/2) phi (16 Zolotarev poles), and the heat
    bath of four sources in one batched call; every solve to the 1e-10 FP64
    true residual.  `extended` adds the FP64 four-source heat bath and the
    mixed forms with FP16S-sloppy refinement."""
    import synth
    c = synth.CONFIGS["c3"]
    dims, mass, n, ns = c["dims"], c["mass"], c["nrhs"], c["nshift"]
    vh = synth.volume(dims) // 2
    F, L = fields
    precs = ("fp64", "fp32", "fp16s") if extended else ("fp64", "fp32")
    g = hisq.Gauge(dims, torch.from_numpy(F).cuda(), torch.from_numpy(L).cuda(), precs)
    for p in precs:
        for k in (1, 4, n, ns):
            hisq.autotune(g, p, k, tune)
    items = []
    srcs = synth.gaussian_source(dims, synth.CFG_IDS["c3"], n, parity=0)
    b = torch.from_numpy(np.concatenate([encode(cb_gather(dims, s_, 0)[0], "fp64") for s_ in srcs])).cuda()
    sb = hisq.spinor_bytes("fp64", vh)
    out = {"workload": f"{'x'.join(map(str, dims))}, m={mass}, tol 1e-10 (FP64 true residual)",
           "long_links_compressed": g.compressed}

    def timed(fn, warm):
        warm()
        torch.cuda.synchronize()
        t1 = time.time()
        r = fn()
        torch.cuda.synchronize()
        return r, time.time() - t1

    def summary(rc, st, wall, k):
        return {"status": rc, "seconds": round(wall, 4), "seconds_per_rhs": round(wall / k, 4),
                "iterations_max": max(v["iterations"] for v in st),
                "true_residual_max": max(v["true_residual"] for v in st)}

    b0 = b[:sb]
    for name, sloppy in (("plain_fp64_1rhs", "fp64"), ("mixed_fp32_1rhs", "fp32")):
        x = torch.zeros_like(b0)
        (rc, st), wall = timed(lambda: hisq.cg_solve(g, mass, 1, b0, x, hisq.solver_params(sloppy_prec=sloppy)),
                               lambda: hisq.cg_solve(g, mass, 1, b0, torch.zeros_like(b0),
                                                     hisq.solver_params(sloppy_prec=sloppy, max_iter=50)))
        out[name] = summary(rc, st, wall, 1)
        items.append((name, srcs[0], _host_solution(dims, x, vh), 0.0))
        log(f"C3 {name}: {wall:.3f} s, {st[0]['iterations']} it, true res {st[0]['true_residual']:.2e}")
    for sl in ("fp32",):
        x = torch.zeros_like(b)
        (rc, st), wall = timed(lambda: hisq.cg_solve(g, mass, n, b, x, hisq.solver_params(sloppy_prec=sl)),
                               lambda: hisq.cg_solve(g, mass, n, b, torch.zeros_like(b),
                                                     hisq.solver_params(sloppy_prec=sl, max_iter=50)))
        key = f"batched_mixed_{sl}_{n}rhs"
        out[key] = summary(rc, st, wall, n)
        items += [(f"{key}[{i}]", srcs[i], _host_solution(dims, x, vh, i), 0.0) for i in range(n)]
        log(f"C3 batched mixed {sl.upper()}, {n} RHS: {wall:.3f} s ({wall / n:.3f} s per RHS), "
            f"max {out[key]['iterations_max']} it, worst true res {out[key]['true_residual_max']:.2e}")
    shifts = [float(v) for v in synth.shifted_ladder(ns)]
    for sl in ("fp64", "fp32"):
        xs = torch.zeros(ns * sb, dtype=torch.uint8, device="cuda")
        prm = hisq.solver_params(sloppy_prec=sl)
        (rc, st), wall = timed(lambda: hisq.multishift_cg(g, mass, shifts, b0, xs, prm),
                               lambda: hisq.multishift_cg(g, mass, shifts, b0, torch.zeros_like(xs),
                                                          hisq.solver_params(sloppy_prec=sl, max_iter=50)))
        ms = summary(rc, st, wall, ns)
        ms["shifts"] = shifts
        items += [(f"multishift_{sl}[{k}]", srcs[0], _host_solution(dims, xs, vh, k), shifts[k]) for k in range(ns)]
        ms["iterations_base"] = st[int(np.argmin(shifts))]["iterations"]
        ms["iterations_per_shift"] = [v["iterations"] for v in st]
        out[f"multishift_{sl}_{ns}shifts"] = ms
        log(f"C3 multi-shift {sl.upper()}, {ns} shifts: {wall:.3f} s, base {ms['iterations_base']} it, "
            f"worst true res {ms['true_residual_max']:.2e}")
    # rooted-staggered pseudofermions for two flavours on [4 m^2, 1.05 x the
    # power-iteration estimate of the top eigenvalue]: heat bath phi = A^(1/4) eta
    # (Remez coefficients), then the action phi^+ A^(-1/2) phi (Zolotarev), which
    # returns |eta|^2 up to the two approximation errors; each with the FP64
    # multi-shift and with the mixed one (FP32 Krylov iteration, FP32-sloppy
    # refinement)
    t1 = time.time()
    lo, hi = hisq.spectral_bounds(g, mass, 100)
    t_bounds = time.time() - t1
    npole = 16
    t1 = time.time()
    h0, hal, hsh, hdelta = hisq.rational_remez(0.25, lo, 1.05 * hi, npole)
    t_remez = time.time() - t1
    a0, al, sh, delta = hisq.zolotarev_inv_sqrt(lo, 1.05 * hi, npole)
    eta2 = float(torch.dot(b0.view(torch.float64), b0.view(torch.float64)))
    phi_one = {}
    # the extended (--c3-solvers) run adds the mixed form with FP16S-sloppy
    # refinement (FP32 Krylov iteration as before)
    hb_precs = ("fp64", "fp32", "fp16s") if extended else ("fp64", "fp32")
    sfx_of = {"fp64": "", "fp32": "_mixed_fp32", "fp16s": "_mixed_fp16s"}
    for sl in hb_precs:
        sfx = sfx_of[sl]
        prm = hisq.solver_params(sloppy_prec=sl)
        warm = hisq.solver_params(sloppy_prec=sl, max_iter=50)
        phi = torch.empty_like(b0)
        (rc, st), wall = timed(lambda: hisq.rational_apply(g, mass, h0, hal, hsh, b0, phi, prm),
                               lambda: hisq.rational_apply(g, mass, h0, hal, hsh, b0, torch.empty_like(b0), warm))
        out[f"heatbath_quarter_root_remez_{npole}poles{sfx}"] = {
            "status": rc, "seconds": round(wall, 4), "remez_seconds": round(t_remez, 4),
            "approximation_rel_error": hdelta, "iterations_base": st[0]["iterations"],
            "true_residual_max": max(v["true_residual"] for v in st)}
        log(f"C3 heat bath A^(1/4) eta ({sl} multi-shift), {npole} Remez poles (rel. error {hdelta:.1e}, "
            f"coefficients {t_remez:.3f} s): {wall:.3f} s, base {st[0]['iterations']} it")
        phi_one[sl] = phi
        y = torch.empty_like(b0)
        (rc, st), wall = timed(lambda: hisq.rational_apply(g, mass, a0, al, sh, phi, y, prm),
                               lambda: hisq.rational_apply(g, mass, a0, al, sh, phi, torch.empty_like(b0), warm))
        action = float(torch.dot(phi.view(torch.float64), y.view(torch.float64)))
        out[f"inv_sqrt_zolotarev_{npole}poles{sfx}"] = {
            "status": rc, "seconds": round(wall, 4), "spectral_bounds": [lo, hi],
            "bounds_seconds": round(t_bounds, 4), "approximation_rel_error": delta,
            "iterations_base": st[0]["iterations"], "true_residual_max": max(v["true_residual"] for v in st),
            "pseudofermion_action": action, "action_over_eta2_minus_1": action / eta2 - 1.0}
        log(f"C3 action phi^+ A^(-1/2) phi ({sl} multi-shift), {npole} Zolotarev poles on [{lo:.2e}, "
            f"{1.05 * hi:.3f}] (rel. error {delta:.1e}): {wall:.3f} s, base {st[0]['iterations']} it; "
            f"S/|eta|^2 - 1 = {action / eta2 - 1:.1e}; bounds {t_bounds:.3f} s")
    # four pseudofermion heat baths in one batched call: the multi-shift
    # iterates the sources in lockstep through the 4-RHS Dslash (FP64, or FP32
    # in the mixed form) and verifies / refines all 4 x 16 (source, pole)
    # systems in one batched CG
    nps = 4
    bq = b[:nps * sb]
    # (the FP64 and FP16S-refinement forms only in the --c3-solvers run: the
    # default run keeps its total time well inside a few minutes)
    for sl in (hb_precs if extended else ("fp32",)):
        sfx = sfx_of[sl]
        phis = torch.empty_like(bq)
        prm = hisq.solver_params(sloppy_prec=sl)
        (rc, st), wall = timed(
            lambda: hisq.rational_apply_batched(g, mass, nps, h0, hal, hsh, bq, phis, prm),
            lambda: hisq.rational_apply_batched(g, mass, nps, h0, hal, hsh, bq, torch.empty_like(bq),
                                                hisq.solver_params(sloppy_prec=sl, max_iter=50)))
        single = out[f"heatbath_quarter_root_remez_{npole}poles{sfx}"]["seconds"]
        ref = phi_one[sl].view(torch.float64)
        d0 = float((phis[:sb].view(torch.float64) - ref).norm() / ref.norm())
        out[f"heatbath_quarter_root_remez_{npole}poles{sfx}_{nps}sources_batched"] = {
            "status": rc, "seconds": round(wall, 4), "seconds_per_source": round(wall / nps, 4),
            "speedup_per_source_vs_one_source": round(single / (wall / nps), 3),
            "iterations_base_max": max(st[j * npole]["iterations"] for j in range(nps)),
            "true_residual_max": max(v["true_residual"] for v in st),
            "source0_rel_diff_vs_one_source_call": d0}
        log(f"C3 heat bath A^(1/4) eta for {nps} sources batched ({sl} multi-shift): {wall:.3f} s, "
            f"{wall / nps:.3f} s per source ({single / (wall / nps):.2f}x one source at a time); "
            f"source 0 differs from the one-source call by {d0:.1e}")
    p1 = out["plain_fp64_1rhs"]["seconds"]
    out["speedup_batched_per_rhs_vs_plain"] = round(p1 / out[f"batched_mixed_fp32_{n}rhs"]["seconds_per_rhs"], 3)
    ms = min((out[f"multishift_{sl}_{ns}shifts"] for sl in ("fp64", "fp32")), key=lambda v: v["seconds"])
    out["speedup_multishift_per_shift_vs_plain"] = round(p1 / ms["seconds_per_rhs"], 3)
    g.close()
    return out, (dims, mass, items)


def run_nn(hisq, torch, fields, npairs=2048, batch=16, epochs=1, lr=3e-3):
    """Train the 1 -> 8 -> 8 -> 1 network on (A v, v) pairs generated on the GPU from
    this gauge field (v Gaussian from a seeded torch generator), then solve one
    Gaussian RHS with plain FP64 CG, mixed FP32 CG and flexible CG with the
    untrained (identity / 6) and the trained network."""
    import synth
    c = synth.CONFIGS["c4"]
    dims, mass = c["dims"], c["mass"]
    vh = synth.volume(dims) // 2
    F, L, U = fields
    g = hisq.Gauge(dims, torch.from_numpy(F).cuda(), torch.from_numpy(L).cuda(), ("fp64", "fp32"))
    hisq.gauge_set_thin(g, torch.from_numpy(np.ascontiguousarray(U)).cuda())
    items = []
    diag = 4 * mass * mass
    chans = (1, 8, 8, 1)
    w0 = np.zeros(9 * (8 + 64 + 8), np.complex128)
    w0[0] = 1.0 / (diag + 6.0)          # layer 1, identity path, channel 0
    w0[9 * 8] = 1.0                     # layer 2, identity path, 0 -> 0
    w0[9 * 8 + 9 * 64] = 1.0            # layer 3, identity path, 0 -> 0
    ident = hisq.Net(g, chans, w0)
    net = hisq.Net(g, chans, w0)
    n6 = 6 * vh                          # floats per FP32 spinor
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2111_10354)
    V = torch.randn(npairs * n6, generator=gen, device="cuda", dtype=torch.float32)
    AV = torch.empty_like(V)
    T = torch.empty(16 * n6, device="cuda", dtype=torch.float32)
    torch.cuda.synchronize()
    t0 = time.time()
    for i in range(0, npairs, 16):
        k = min(16, npairs - i)
        vv, aa = V[i * n6:(i + k) * n6], AV[i * n6:(i + k) * n6]
        hisq.dslash_multi_rhs(g, 1, "fp32", k, vv, T[:k * n6])
        hisq.dslash_multi_rhs(g, 0, "fp32", k, T[:k * n6], aa, diag=[diag] * k, y=vv)
    torch.cuda.synchronize()
    t_pairs = time.time() - t0
    del T
    l0 = net.loss_grad(batch, AV[:batch * n6], V[:batch * n6], want_grad=False)[0]
    steps = epochs * (npairs // batch)
    torch.cuda.synchronize()
    t0 = time.time()
    for s in range(steps):
        i = s % (npairs // batch)
        net.train_step(batch, AV[i * batch * n6:(i + 1) * batch * n6], V[i * batch * n6:(i + 1) * batch * n6], lr)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    l1 = net.loss_grad(batch, AV[:batch * n6], V[:batch * n6], want_grad=False)[0]
    log(f"network: {npairs} pairs in {t_pairs:.2f} s, {steps} Adam steps in {t_train:.1f} s, "
        f"loss {l0:.4f} -> {l1:.4f}")
    del V, AV
    torch.cuda.empty_cache()
    # cost of one network pass against one FP32 application of A
    r = torch.randn(n6, generator=gen, device="cuda", dtype=torch.float32)
    z, t1 = torch.empty_like(r), torch.empty_like(r)
    hisq.precond_apply(g, net, r, z)
    ms_nn = time_launches(lambda: hisq.precond_apply(g, net, r, z), 20, 3)
    ms_a = time_launches(lambda: (hisq.dslash_multi_rhs(g, 1, "fp32", 1, r, t1),
                                  hisq.dslash_multi_rhs(g, 0, "fp32", 1, t1, z, diag=[diag], y=r)), 20, 3)
    b = synth.gaussian_source(dims, synth.CFG_IDS["c4"], 1, parity=0)[0]
    bd = torch.from_numpy(encode(cb_gather(dims, b, 0)[0], "fp64")).cuda()
    out = {"workload": f"{'x'.join(map(str, dims))}, m={mass}, network 1-8-8-1 (BF16 MFMA mixing), "
                       f"{npairs} (A v, v) pairs, batch {batch}, {epochs} epoch(s), 1 Gaussian RHS, tol 1e-10",
           "pairs_seconds": round(t_pairs, 3), "train_seconds": round(t_train, 2), "train_steps": steps,
           "loss_start": round(l0, 5), "loss_trained": round(l1, 5),
           "ms_network_pass": round(ms_nn, 4), "ms_A_fp32": round(ms_a, 4), "solves": {}}
    for name, kw in (("plain_fp64", {}), ("mixed_fp32", {"sloppy_prec": "fp32"}),
                     ("fcg_untrained", {"precond": ident}), ("fcg_trained", {"precond": net})):
        x = torch.zeros_like(bd)
        hisq.cg_solve(g, mass, 1, bd, x, hisq.solver_params(max_iter=50, **kw))
        x.zero_()
        torch.cuda.synchronize()
        t1 = time.time()
        rc, st = hisq.cg_solve(g, mass, 1, bd, x, hisq.solver_params(**kw))
        wall = time.time() - t1
        out["solves"][name] = {"status": rc, "seconds": round(wall, 4), "iterations": st[0]["iterations"],
                               "fallback_used": st[0]["fallback_used"], "true_residual": st[0]["true_residual"]}
        items.append((name, b, _host_solution(dims, x, vh), 0.0))
        log(f"{name}: {wall:.3f} s, {st[0]['iterations']} it, true res {st[0]['true_residual']:.2e}")
    sv = out["solves"]
    out["iterations_trained_over_plain"] = round(sv["fcg_trained"]["iterations"] / sv["plain_fp64"]["iterations"], 4)
    out["iterations_trained_over_untrained"] = round(sv["fcg_trained"]["iterations"] /
                                                     sv["fcg_untrained"]["iterations"], 4)
    ident.close()
    net.close()
    g.close()
    return out, (dims, mass, items)


def run_c5_solve(hisq, torch, tune, dims, F, L, gauge=None, plain_rhs=1, with_fp16s=False):
    """(D^+D + 4m^2) x = b on 96^3 x 24, m = 0.002, 4 Gaussian RHS, tol 1e-10 on the
    FP64 true residual.  Plain form: FP64 CG one RHS at a time (timed on the
    first `plain_rhs` RHS; the 4-RHS total is that time per RHS x 4, marked as
    such).  Chosen form: the 4 RHS batched through the multi-RHS Dslash with FP32
    (or, on request, also FP16S) sloppy iterations and FP64 reliable updates.
    `gauge`: a handle of these links with FP64, FP32 and FP16 copies (else one
    is built here)."""
    import synth
    c = synth.CONFIGS["c5"]
    mass, n = c["mass"], c["nrhs"]
    vh = synth.volume(dims) // 2
    g = gauge
    if g is None:
        fd, ld = torch.from_numpy(F).cuda(), torch.from_numpy(L).cuda()
        g = hisq.Gauge(dims, fd, ld, ("fp64", "fp32", "fp16s"))
        torch.cuda.synchronize()
        del fd, ld
        torch.cuda.empty_cache()
    for p in ("fp64", "fp32") + (("fp16s",) if with_fp16s else ()):
        for k in (1, n):
            hisq.autotune(g, p, k, tune)
    srcs = synth.gaussian_source(dims, synth.CFG_IDS["c5"], n, parity=0)
    b = torch.from_numpy(np.concatenate([encode(cb_gather(dims, s_, 0)[0], "fp64") for s_ in srcs])).cuda()
    sb = hisq.spinor_bytes("fp64", vh)
    out = {"workload": f"{'x'.join(map(str, dims))}, m={mass}, {n} Gaussian RHS, tol 1e-10 (FP64 true residual)",
           "long_links_compressed": g.compressed}
    items = []
    # plain form
    per = []
    for i in range(plain_rhs):
        bi = b[i * sb:(i + 1) * sb]
        x = torch.zeros_like(bi)
        torch.cuda.synchronize()
        t1 = time.time()
        rc, st = hisq.cg_solve(g, mass, 1, bi, x, hisq.solver_params(sloppy_prec="fp64", graph_chunk=25))
        wall = time.time() - t1
        per.append({"status": rc, "seconds": round(wall, 3), "iterations": st[0]["iterations"],
                    "true_residual": st[0]["true_residual"]})
        items.append((f"plain_fp64[{i}]", srcs[i], _host_solution(dims, x, vh), 0.0))
        log(f"C5 plain FP64 RHS {i}: {wall:.1f} s, {st[0]['iterations']} it, true res {st[0]['true_residual']:.2e}")
        del x
    mean = sum(r["seconds"] for r in per) / len(per)
    out["plain_fp64"] = {"per_rhs": per, "seconds_per_rhs": round(mean, 3),
                         "seconds_4rhs": round(mean * n, 3),
                         "note": f"timed on {plain_rhs} of {n} RHS; the {n}-RHS total is the per-RHS time x {n} "
                                 "(extrapolated)"}
    forms = (("batched_mixed_fp32", "fp32"),) + ((("batched_mixed_fp16s", "fp16s"),) if with_fp16s else ())
    for name, sloppy in forms:
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t1 = time.time()
        rc, st = hisq.cg_solve(g, mass, n, b, x, hisq.solver_params(sloppy_prec=sloppy, graph_chunk=25))
        wall = time.time() - t1
        out[name] = {"status": rc, "seconds_4rhs": round(wall, 3), "seconds_per_rhs": round(wall / n, 3),
                     "iterations": [s_["iterations"] for s_ in st],
                     "true_residual": [s_["true_residual"] for s_ in st]}
        items += [(f"{name}[{i}]", srcs[i], _host_solution(dims, x, vh, i), 0.0) for i in range(n)]
        log(f"C5 {name}: {wall:.1f} s for {n} RHS, iterations {[s_['iterations'] for s_ in st]}, "
            f"worst true res {max(s_['true_residual'] for s_ in st):.2e}")
        del x
    best = min((f for f, _ in forms), key=lambda k: out[k]["seconds_4rhs"] if out[k]["status"] == 0 else 1e30)
    out["chosen"] = best
    out["speedup_chosen_vs_plain"] = round(out["plain_fp64"]["seconds_4rhs"] / out[best]["seconds_4rhs"], 3)
    if gauge is None:
        g.close()
    return out, (dims, mass, items)


if __name__ == "__main__":
    main()
