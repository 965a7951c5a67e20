"""Benchmark: SHT synthesis + analysis pairs/s at l = 1024 with 64 complex fields.

One step = synthesis of a batch of F fields (coefficients -> 2l x 4l grid) followed by
analysis of that grid back to coefficients, on one MI355X, with every input already in
device memory.  value = F * steps / (timed seconds) for the split-FP32 butterfly (the
--precision default); the plain FP64 butterfly and plain FP32 are timed the same way in the
same run and reported under "variants", with the per-field relative l2 error of each
variant against the FP64 butterfly on the full batch ("err_vs_fp64").  The plan precompute
is excluded and reported as t_plan_s.

The JSON line also carries
 * roofline: the stage with the largest share of the timed kernel time, its algorithmic
   flops (factor entries x R x 2) or bytes per launch divided by its mean launch time as
   measured with HIP events inside the library on the launch stream, against the MI355X
   peak of the unit that bounds it;
 * cpu_baseline: the CPU oracle timed on a bounded sample of the same workload (a subset
   of orders, a subset of fields), extrapolated by the exact operation counts, with the
   GPU-vs-oracle error on that sample.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SHT synth+analysis pairs/s at l=1024, 64 fields: split-FP32 vs FP64, 1e-9 err"
PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "hbm": 8.0e12}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--per-field-steps", type=int, default=1,
                    help="steps (each F single-field pairs) for the per-field FP64 variant")
    ap.add_argument("--l", type=int, default=1024)
    ap.add_argument("--fields", type=int, default=64)
    ap.add_argument("--precision", default="split32", choices=["fp64", "split32", "fp32"])
    ap.add_argument("--no-variants", action="store_true", help="time only --precision")
    ap.add_argument("--leaf-width", type=int, default=64)
    ap.add_argument("--eps", type=float, default=1e-12)
    ap.add_argument("--power", type=float, default=1.5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-orders", type=int, default=48)
    ap.add_argument("--cpu-fields", type=int, default=4,
                    help="fields in the oracle sample (a multiple of 4 for the matrix-core variants)")
    ap.add_argument("--workload", default="metric", choices=["metric", "mixed", "single"],
                    help="metric: the l=1024, 64-field line; mixed: 96 requests of mixed bandlimits "
                         "through the batched persistent launch, beside one call per request; single: "
                         "one complex field at l=256 in FP64 (the factor-streaming regime)")
    ap.add_argument("--mixed-bandlimits", default="32,64,128,256,512,1024",
                    help="bandlimits of the mixed workload (uniform draw); the full set 64..2048 needs "
                         "about 210 GB for its inputs and outputs alone")
    ap.add_argument("--no-gemm-baseline", action="store_true",
                    help="skip the direct FP64 Legendre GEMM (library DGEMM on dense Q) comparison")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 2 GiB device-to-device copy (HBM counter calibration)")
    return ap.parse_args()


def rel_err_per_field(a, b):
    import torch

    F = a.shape[0]
    d = (a - b).reshape(F, -1)
    r = b.reshape(F, -1)
    return (torch.linalg.norm(d, dim=1) / torch.linalg.norm(r, dim=1)).cpu().numpy()


def cpu_baseline(plan, args, beta_np, grid_seed_np):
    """Time the oracle on a sample of orders and fields; extrapolate to the full batch."""
    import numpy as np
    import torch
    from threadpoolctl import threadpool_info

    import oracle

    l, F = args.l, args.fields
    L2 = 2 * l
    Fs = min(args.cpu_fields, F)
    norders = max(2, min(args.cpu_orders, L2))
    sample = sorted(set(int(round(v)) for v in np.linspace(0, L2 - 1, norders)))
    ms = np.abs(__import__("sht_synthetic").orders_canonical(l))
    mask = np.isin(ms, sample)
    beta_s = np.where(mask[None, :], beta_np[:Fs], 0.0)

    # oracle: synthesis and analysis of the sampled orders (Legendre sums) ...
    t0 = time.perf_counter()
    f_ref = oracle.synth(beta_s, l, orders=sample)
    t1 = time.perf_counter()
    a_ref = oracle.analyze_orders(grid_seed_np[:Fs], l, sample)
    t2 = time.perf_counter()
    # ... and the longitude FFTs of the sampled fields (both directions)
    g = np.fft.ifft(f_ref, axis=-1)
    g = np.fft.fft(g, axis=-1)
    t3 = time.perf_counter()
    # Legendre cost of an order is proportional to its degree count 2l - |m| (both signs)
    w_all = sum((L2 - m) * (1 if m == 0 else 2) for m in range(L2))
    w_s = sum((L2 - m) * (1 if m == 0 else 2) for m in sample)
    # synth() and analyze_orders() each include one FFT pass over Fs fields; remove it
    t_fft_pair = t3 - t2
    t_leg = max(1e-9, (t1 - t0) + (t2 - t1) - t_fft_pair)
    t_full = (t_leg * w_all / w_s + t_fft_pair) * (F / Fs)

    # GPU on the same sampled inputs (outside the timed region), every variant
    dev_b = torch.from_numpy(np.ascontiguousarray(beta_s)).to("cuda")
    dev_g = torch.from_numpy(np.ascontiguousarray(grid_seed_np[:Fs])).to("cuda")
    a_ref = a_ref[:, mask]
    errs = {}
    for prec in dict.fromkeys([args.precision, "fp64"]):
        f_gpu = plan.synth(dev_b, precision=prec).cpu().numpy()
        a_gpu = plan.analyze(dev_g, precision=prec).cpu().numpy()[:, mask]
        errs[prec] = {
            "synth": [float(np.linalg.norm(f_gpu[i] - f_ref[i]) / np.linalg.norm(f_ref[i])) for i in range(Fs)],
            "analysis": [float(np.linalg.norm(a_gpu[i] - a_ref[i]) / np.linalg.norm(a_ref[i]))
                         for i in range(Fs)],
        }
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    return {
        "value": F / t_full,
        "unit": "pairs/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"{len(sample)} of {L2} orders ({sample[0]}..{sample[-1]}), {Fs} of {F} fields; "
                  f"measured {t3 - t0:.1f} s, extrapolated by degree counts to {t_full:.0f} s per batch",
        "gpu_rel_err_vs_oracle": errs,
    }


def time_pairs(plan, prec, beta, grid, back, steps, warmup, profile=False):
    """Warm up, then time `steps` synthesis+analysis pairs with events on the current stream.

    Returns (total ms, per-step ms list, wall seconds, profile or None)."""
    import torch

    for _ in range(warmup):
        plan.synth(beta, out=grid, precision=prec)
        plan.analyze(grid, out=back, precision=prec)
    torch.cuda.synchronize()
    if profile:
        plan.profile_reset()
        plan.profile(True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev[0].record()
    for i in range(steps):
        plan.synth(beta, out=grid, precision=prec)
        plan.analyze(grid, out=back, precision=prec)
        ev[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    prof = None
    if profile:
        plan.profile(False)
        prof = plan.profile_read()
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return ev[0].elapsed_time(ev[steps]), per, wall, prof


def time_per_field(plan, beta, steps):
    """Plain FP64 butterfly one field at a time (R = 4 columns: the vector kernels)."""
    import torch

    F = beta.shape[0]
    g1 = torch.empty((1,) + plan.grid_shape, dtype=torch.complex128, device="cuda")
    b1 = torch.empty((1, beta.shape[1]), dtype=torch.complex128, device="cuda")
    fields = [beta[f:f + 1] for f in range(F)]
    plan.synth(fields[0], out=g1, precision="fp64")
    plan.analyze(g1, out=b1, precision="fp64")
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        for f in range(F):
            plan.synth(fields[f], out=g1, precision="fp64")
            plan.analyze(g1, out=b1, precision="fp64")
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


POLAR_TRIM = 1e-15  # |Q| below this on a whole node row: the row is left out of the trimmed GEMM


def polar_rows(Q, chunk=256):
    """Per (m, p): the number of leading nodes (ascending x, equator first) up to the last
    node whose row of Q^(m,p) (stored transposed, n x l) has an entry above POLAR_TRIM.
    Towards the pole P^m_k decays like (1 - x^2)^(m/2), so the rows past that node are
    negligible at high order."""
    import torch

    npair, _, l = Q.shape
    idx = torch.arange(1, l + 1, device=Q.device)
    rows = []
    for a in range(0, npair, chunk):
        big = Q[a:a + chunk].abs().amax(dim=1) > POLAR_TRIM  # (pairs, l)
        rows.append(torch.where(big, idx, torch.zeros_like(idx)).amax(dim=1))
    return [int(r) for r in torch.cat(rows).tolist()]


def gemm_runs(ncols, rows, run=128):
    """Runs of `run` consecutive pairs, each padded to its largest column count and node
    count; runs with no work are dropped."""
    out = []
    for a in range(0, len(ncols), run):
        b = min(len(ncols), a + run)
        n, r = max(ncols[a:b]), max(rows[a:b])
        if n > 0 and r > 0:
            out.append((a, b, n, r))
    return out


def gemm_baseline(plan, l, R, steps):
    """Direct FP64 Legendre step on the library DGEMM (torch.bmm): every dense Q^(m,p),
    generated on the device by the plan's column kernel, applied to R columns in synthesis
    (Q X) and in analysis (Q^T Y).  Pairs are taken in runs of 128 consecutive (m, p), each
    run padded to its largest column count n_p.  Timed twice: over all l nodes, and with
    polar trimming (each run restricted to the nodes where some Q^(m,p) of the run is above
    POLAR_TRIM).  Returns times per direction."""
    import torch

    npair = 4 * l
    ncols = [max(0, (2 * l - mp // 2 - mp % 2 + 1) // 2) for mp in range(npair)]
    Q = torch.zeros((npair, l, l), dtype=torch.float64, device="cuda")
    for mp0 in range(0, npair, 256):
        plan.dense_q(Q[mp0:], mp0, min(256, npair - mp0))
    g = torch.Generator(device="cuda").manual_seed(0)
    Xt = torch.randn((npair, R, l), dtype=torch.float64, device="cuda", generator=g)
    Y = torch.randn((npair, l, R), dtype=torch.float64, device="cuda", generator=g)

    def timed(runs):
        def synth():
            for a, b, n, r in runs:
                torch.bmm(Xt[a:b, :, :n], Q[a:b, :n, :r])

        def analysis():
            for a, b, n, r in runs:
                torch.bmm(Q[a:b, :n, :r], Y[a:b, :r])

        res = {}
        for name, fn in (("synth", synth), ("analysis", analysis)):
            fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            res[name + "_ms"] = e0.elapsed_time(e1) / steps
        return res

    runs = gemm_runs(ncols, [l] * npair)
    out = timed(runs)
    dense = sum(l * n for n in ncols)
    padded = sum((b - a) * r * n for a, b, n, r in runs)
    out.update({"dense_entries": dense, "padded_entries": padded,
                "tflops_synth": 2.0 * padded * R / (out["synth_ms"] / 1e3) / 1e12,
                "tflops_analysis": 2.0 * padded * R / (out["analysis_ms"] / 1e3) / 1e12})
    try:
        rows = polar_rows(Q)
        truns = gemm_runs(ncols, rows)
        tr = timed(truns)
        out["polar_trimmed"] = {
            "threshold": POLAR_TRIM, "synth_ms": tr["synth_ms"], "analysis_ms": tr["analysis_ms"],
            "entries": sum(r * n for r, n in zip(rows, ncols)),
            "padded_entries": sum((b - a) * r * n for a, b, n, r in truns)}
    except Exception as exc:  # a comparison only: never let it end the run
        out["polar_trimmed"] = {"error": repr(exc)}
    del Q, Xt, Y
    torch.cuda.empty_cache()
    return out


def stage_totals(prof, steps):
    """Per butterfly step: the size-class launches ("level2.c0", "level2.c1") summed."""
    import re

    out = {}
    for k, v in prof.items():
        key = re.sub(r"\.c\d+/", "/", k)
        out[key] = out.get(key, 0.0) + v["ms"] / steps
    return dict(sorted(out.items()))


def measured_traffic(launch):
    """HBM bytes per launch from the committed counter summary, if it was taken on the kernel
    source that is built now (else None)."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    ent = rec.get("launches", {}).get(launch)
    src = os.path.join(ROOT, rec.get("kernel_source", ""))
    if ent is None or not os.path.exists(src):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec.get("kernel_source_sha256"):
        return None
    return ent["bytes"]


def roofline(prof, ms_total, precision):
    """The single kernel launch with the largest share of the timed kernel time."""
    name, rec = max(prof.items(), key=lambda kv: kv[1]["ms"])
    mean_s = rec["ms"] / rec["launches"] / 1e3
    flops_rate = rec["flops"] / mean_s
    bytes_rate = rec["bytes"] / mean_s
    peak_f = PEAK["fp64"] if precision == "fp64" else PEAK["fp32"]
    if rec["flops"] > 0 and rec["flops"] / max(rec["bytes"], 1.0) > peak_f / PEAK["hbm"]:
        roof = {"bound": "mfma", "achieved": flops_rate / 1e12, "peak": peak_f / 1e12,
                "unit": "TFLOP/s", "frac": flops_rate / peak_f}
    else:
        roof = {"bound": "hbm", "achieved": bytes_rate / 1e9, "peak": PEAK["hbm"] / 1e9,
                "unit": "GB/s", "frac": bytes_rate / PEAK["hbm"]}
    roof.update({"kernel": name, "mean_launch_ms": mean_s * 1e3, "launches": rec["launches"],
                 "flops_per_launch": rec["flops"], "bytes_per_launch": rec["bytes"],
                 "traffic": measured_traffic(name), "share_of_step": rec["ms"] / ms_total})
    return roof


def mixed(args):
    """96 requests, bandlimits uniform over a set, 1..16 complex fields each (default_rng(0));
    one synthesis batch and one analysis batch (persistent launch, graph, tuned) per step,
    against one synth + analyze call per request."""
    import numpy as np
    import torch

    import sht_synthetic as syn
    from paper_0910_5435_amd import Batch, Plan

    bls = [int(v) for v in args.mixed_bandlimits.split(",")]
    rng = np.random.default_rng(0)
    ls = rng.choice(bls, 96)
    fs = rng.integers(1, 17, 96)
    t0 = time.perf_counter()
    plans = {l: Plan(l, eps=args.eps, leaf_width=min(args.leaf_width, max(4, l // 2)))
             for l in sorted(set(int(v) for v in ls))}
    t_plan = time.perf_counter() - t0
    print(f"# mixed: plans {sorted(plans)} in {t_plan:.1f} s", file=sys.stderr, flush=True)
    reqs = []
    for i, (l, F) in enumerate(zip(ls, fs)):
        l, F = int(l), int(F)
        P = plans[l]
        c = torch.from_numpy(syn.coefficients(l, F, seed=i, power=args.power)).cuda()
        g = torch.empty((F, 2 * l, 4 * l), dtype=torch.complex128, device="cuda")
        b = torch.empty_like(c)
        reqs.append((P, c, g, b))
    fields = int(fs.sum())
    out = {"metric": "mixed-request SHT synth+analysis pairs/s", "unit": "pairs/s",
           "higher_is_better": True, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "data": "synthetic",
           "config": {"workload": f"96 requests, l uniform over {bls}, 1..16 complex fields each "
                                  f"({fields} fields), coefficients CN(0,1)/(1+k)^{args.power}",
                      "requests": 96, "fields": fields, "eps": args.eps},
           "t_plan_s": t_plan}
    for prec in ("split32", "fp64"):
        bs = Batch([(P, c, g) for (P, c, g, _) in reqs], op="synth", precision=prec)
        ba = Batch([(P, g, b) for (P, _, g, b) in reqs], op="analyze", precision=prec)
        tuned = (bs.tune(reps=2), ba.tune(reps=2))
        for _ in range(args.warmup):
            bs.run()
            ba.run()
        bs.check()
        ba.check()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            bs.run()
            ba.run()
        e1.record()
        bs.check()
        ba.check()
        ms = e0.elapsed_time(e1) / args.steps
        err = max(float(((b - c).abs().pow(2).sum(dim=1).sqrt() / c.abs().pow(2).sum(dim=1).sqrt()).max())
                  for (_, c, _, b) in reqs)
        # one synth + analyze call per request, same stream, same precision where it runs
        # (split needs 4 | fields; those requests fall back to FP64 calls here)
        for (P, c, g, b) in reqs:
            p1 = prec if (c.shape[0] % 4 == 0 or prec == "fp64") else "fp64"
            P.synth(c, out=g, precision=p1)
            P.analyze(g, out=b, precision=p1)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            for (P, c, g, b) in reqs:
                p1 = prec if (c.shape[0] % 4 == 0 or prec == "fp64") else "fp64"
                P.synth(c, out=g, precision=p1)
                P.analyze(g, out=b, precision=p1)
        e1.record()
        torch.cuda.synchronize()
        ms_seq = e0.elapsed_time(e1) / args.steps
        out[prec] = {"batched_pairs_per_s": fields / (ms / 1e3), "batched_ms_per_step": ms,
                     "per_request_pairs_per_s": fields / (ms_seq / 1e3), "per_request_ms_per_step": ms_seq,
                     "round_trip_rel_err_max": err, "tuned": {"synth": tuned[0], "analysis": tuned[1]},
                     "batch_info": {"synth": bs.info(), "analysis": ba.info()}}
        print(f"# mixed {prec}: batched {ms:.1f} ms/step, per request {ms_seq:.1f} ms/step, rt {err:.2e}",
              file=sys.stderr, flush=True)
        bs.close()
        ba.close()
    out["value"] = out["split32"]["batched_pairs_per_s"]
    out["dtype"] = "f32"
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design note, not built.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "mixed":
        return mixed(args)
    metric = METRIC
    if args.workload == "single":
        # one complex field, l = 256, FP64 butterfly (vector kernels at R = 4): the oracle runs
        # on every order
        args.l, args.fields, args.precision, args.no_variants = 256, 1, "fp64", True
        args.power, args.eps, args.cpu_fields, args.cpu_orders = 1.0, 1e-13, 1, 512
        metric = "SHT synth+analysis pairs/s at l=256, 1 field, FP64 butterfly"
    import numpy as np
    import torch

    import sht_synthetic as syn
    from paper_0910_5435_amd import Plan

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    l, F = args.l, args.fields
    if args.calibrate_copy:
        # plain copy of known size: 2 GiB read + 2 GiB written per launch
        a = torch.empty(2 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    t0 = time.perf_counter()
    plan = Plan(l, eps=args.eps, leaf_width=args.leaf_width, precision=args.precision)
    t_plan = time.perf_counter() - t0
    st = plan.stats()
    print(f"# plan l={l} eps={args.eps} C={args.leaf_width}: {t_plan:.1f} s, k_max={st['k_max']} "
          f"k_avg={st['k_avg']:.1f} factors={st['factor_entries']:.3e} (columns {st['t_columns_s']:.1f} s, "
          f"IDs {st['t_compress_s']:.1f} s)", file=sys.stderr, flush=True)

    beta_np = syn.coefficients(l, F, seed=0, power=args.power)
    beta = torch.from_numpy(beta_np).to("cuda")
    grid = torch.empty((F, 2 * l, 4 * l), dtype=torch.complex128, device="cuda")
    back = torch.empty_like(beta)

    ms_total, per_step, wall, prof = time_pairs(plan, args.precision, beta, grid, back, args.steps,
                                                args.warmup, profile=True)
    ms_step = ms_total / args.steps
    value = F * args.steps / (ms_total / 1e3)
    err_rt = rel_err_per_field(back, beta)
    print(f"# {args.precision}: {value:.1f} pairs/s, {ms_step:.2f} ms/step", file=sys.stderr, flush=True)

    variants = {}
    if not args.no_variants:
        for prec in ("fp64", "split32", "fp32"):
            if prec == args.precision:
                continue
            ms_v, per_v, _, prof_v = time_pairs(plan, prec, beta, grid, back, args.steps, args.warmup,
                                                profile=prec == "fp64")
            variants[prec] = {"value": F * args.steps / (ms_v / 1e3), "ms_per_step": ms_v / args.steps,
                              "ms_per_step_median": float(np.median(per_v))}
            if prof_v:
                variants[prec]["stages_ms_per_step"] = stage_totals(prof_v, args.steps)
            print(f"# {prec}: {variants[prec]['value']:.1f} pairs/s", file=sys.stderr, flush=True)
        if args.per_field_steps > 0:
            ms_pf = time_per_field(plan, beta, args.per_field_steps)
            variants["fp64_per_field"] = {"value": F * args.per_field_steps / (ms_pf / 1e3),
                                          "ms_per_step": ms_pf / args.per_field_steps,
                                          "note": f"{F} single-field calls per direction per step"}
            print(f"# fp64 per field: {variants['fp64_per_field']['value']:.1f} pairs/s", file=sys.stderr,
                  flush=True)

    gemm = None
    if not args.no_gemm_baseline and ("fp64" in variants or args.precision == "fp64"):
        gemm = gemm_baseline(plan, l, 4 * F, max(2, min(args.steps, 5)))
        st64 = variants["fp64"]["stages_ms_per_step"] if "fp64" in variants else stage_totals(prof, args.steps)
        bf = {d: sum(v for k, v in st64.items() if k.startswith(d + ".") and ".fft/" not in k)
              for d in ("synth", "analysis")}
        fft = sum(v for k, v in st64.items() if ".fft/" in k)
        gemm["butterfly_fp64_legendre_ms"] = bf
        gemm["pairs_per_s_with_fft"] = F / ((gemm["synth_ms"] + gemm["analysis_ms"] + fft) / 1e3)
        print(f"# dense DGEMM Legendre: synth {gemm['synth_ms']:.1f} ms, analysis {gemm['analysis_ms']:.1f} ms "
              f"(butterfly FP64 {bf['synth']:.1f} / {bf['analysis']:.1f} ms)", file=sys.stderr, flush=True)
        pt = gemm["polar_trimmed"]
        if "error" not in pt:
            print(f"# dense DGEMM Legendre, polar-trimmed ({pt['entries'] / gemm['dense_entries']:.2f} of the "
                  f"entries): synth {pt['synth_ms']:.1f} ms, analysis {pt['analysis_ms']:.1f} ms",
                  file=sys.stderr, flush=True)

    # per-field error of each precision against the FP64 butterfly on the full batch: synthesis
    # of the bench coefficients, and analysis of the FP64 grid
    err64 = {}
    g64 = plan.synth(beta, precision="fp64")
    b64 = plan.analyze(g64, precision="fp64")
    for prec in ([args.precision] if args.no_variants else ["split32", "fp32"]):
        if prec == "fp64":
            continue
        es = rel_err_per_field(plan.synth(beta, out=grid, precision=prec), g64)
        ea = rel_err_per_field(plan.analyze(g64, out=back, precision=prec), b64)
        err64[prec] = {"synth_max": float(es.max()), "synth_median": float(np.median(es)),
                       "analysis_max": float(ea.max()), "analysis_median": float(np.median(ea))}
    del g64, b64
    torch.cuda.synchronize()

    out = {
        "metric": metric,
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_median": float(np.median(per_step)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "split32": "f32", "fp32": "f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"SHT synthesis+analysis, l={l} (degrees 0..{2 * l - 1}), {F} complex "
                               f"fields, grid {2 * l}x{4 * l}, coefficients CN(0,1)/(1+k)^{args.power}",
                   "l": l, "fields": F, "precision": args.precision, "leaf_width": args.leaf_width,
                   "eps": args.eps},
        "roofline": roofline(prof, ms_total, args.precision),
        "variants": variants,
        "dense_gemm_fp64": gemm,
        "err_vs_fp64": err64,
        "round_trip_rel_err_max": float(np.max(err_rt)),
        "t_plan_s": t_plan,
        "plan": {k: st[k] for k in ("k_max", "k_avg", "k_sd", "factor_entries", "dense_entries",
                                    "m_max_words", "device_bytes", "t_columns_s", "t_compress_s",
                                    "max_abs_t")},
        "wall_s_timed": wall,
        "stages_ms_per_step": stage_totals(prof, args.steps),
        "launches_ms_per_step": {k: v["ms"] / args.steps for k, v in sorted(prof.items())},
    }
    if not args.no_cpu_baseline:
        grid_seed = syn.grid(l, min(args.cpu_fields, F), seed=1)
        out["cpu_baseline"] = cpu_baseline(plan, args, beta_np, grid_seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
