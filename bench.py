"""Benchmark of the encrypted 1:N match on one MI355X.

Workload: the face-scale gallery (N = 2^16, eight 50-bit chain primes, two
special primes, dnum = 4; 6,144 L2-normalised 128-dim templates packed into
24 ciphertexts), one encrypted query.  The parts count k (1, 2, 4, 8, 16) and
the Alg. 2 schedule are swept briefly and the fastest is timed.  A step is one
whole server-side match (Alg. 1 expansion when k > 1, Alg. 2 on every group,
output level drop) with the query and the gallery already resident in HBM.

Output: one JSON line (see the keys below); a roofline entry for the kernel
with the most device time, from HIP events on the launch stream over the timed
region; and a bounded sample of the CPU oracle on the host cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Modular products per second the VALU can issue at most, reported beside the
# HBM figure.  Residues (q < 2^51) are carried in FP64, which CDNA4 issues at
# one operation per lane per clock: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz =
# 39.32 T FP64 operations/s (the 78.6 TFLOP/s vector figure counts an FMA as
# two).  A butterfly (or a multiply-accumulate of the key products) needs at
# least 8 of them: the exact product a*w - round(a*w/q)*q (multiply, FMA for
# the low half, multiply for the quotient, round, FMA, add) and two adds.
# Peak: 39.32e12 / 8 = 4.915 T/s.  Every kernel of the match moves at least
# one 8-byte word per such operation, below the 5 operations per byte at which
# the FP64 VALU would bind before HBM, so the roofline is the HBM one.
ALU_PEAK_GMODMUL = 39.3216e3 / 8.0
# HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE counter runs (scaled by
# a 1 GiB device copy: x2.0 for FETCH_SIZE, x1.0 for WRITE_SIZE), kept with
# the sha256 of the kernel source they were taken on and the workload; the
# figure is reported only while both still match.
TRAFFIC = {
    # the face match at k = 4, S2 + minimum level + hoisted: the grouped hoisted
    # key inner product, as the autotuner's two usual variants build it
    ("k_kip_hoist_zb<1, 3, 4>", "k4_S2+levelmin+hoist"): {
        "kernels_sha256": "1f77b813cb8904ca6851426e9c82c0de83ce7c2c575bbc42c828d5f5647dcddd",
        "algorithmic_bytes_per_launch": 180355072, "bytes_per_launch": 207849277},
    ("k_kip_hoist_zb<1, 2, 4>", "k4_S2+levelmin+hoist"): {
        "kernels_sha256": "1f77b813cb8904ca6851426e9c82c0de83ce7c2c575bbc42c828d5f5647dcddd",
        "algorithmic_bytes_per_launch": 180355072, "bytes_per_launch": 228512294},
}


def kernels_sha256():
    import hashlib
    path = os.path.join(ROOT, "paper_2408_06167_amd", "csrc", "kernels.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_for(kernel, cfg, algorithmic_bytes_per_launch):
    """Counter-measured HBM bytes per launch, or None when the kernels, the
    workload or the launch mix differ from the counter runs."""
    t = TRAFFIC.get((kernel, cfg))
    if t is None or t["kernels_sha256"] != kernels_sha256():
        return None
    if abs(algorithmic_bytes_per_launch / t["algorithmic_bytes_per_launch"] - 1) > 1e-3:
        return None
    return t["bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--k", type=int, default=0, help="parts; 0 sweeps 1..16")
    ap.add_argument("--schedule", type=int, default=0, help="1 or 2; 0 sweeps both")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle sample")
    ap.add_argument("--no-profile", action="store_true", help="no per-kernel events")
    ap.add_argument("--eager", action="store_true", help="launch kernels one by one (no HIP graphs)")
    ap.add_argument("--no-ci", action="store_true", help="skip the conjugate-invariant ring figure")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the compressed, conjugate-invariant and other-workload figures (profiling runs)")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the fingerprint, batched and serving summaries")
    ap.add_argument("--workload", default="face", choices=["face", "fingerprint", "batch", "serve", "copy", "ntt"],
                    help="face: 6,144 x 128-dim (default); fingerprint: 1,048,576 x 16-dim; "
                         "batch: mixed shapes, batched vs per-pair; serve: Poisson arrivals; "
                         "copy: 1 GiB device copy (counter calibration); ntt: batched NTT throughput")
    ap.add_argument("--tuning", default="",
                    help="fixed knobs group_chunk,kip_variant,ntt_row_views,kip_order,fused_occupancy"
                         "[,column_sources] instead of the autotuner (profiler runs that must launch the same "
                         "kernels)")
    ap.add_argument("--scale", type=float, default=1.0, help="gallery size factor for batch/serve")
    ap.add_argument("--rates", default="50,100,200,500,1000,2000", help="serve: arrival rates (queries/s)")
    ap.add_argument("--requests", type=int, default=200, help="serve: requests per rate")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.workload != "face":
        import bench_workloads
        bench_workloads.run(args)
        return
    import torch
    import paper_2408_06167_amd as bm
    from workloads import face_gallery

    d, seed, n_tmpl = 128, 0xB11D, 6144
    w = face_gallery(seed=2, d=d, n=n_tmpl)
    X, q = w["gallery"], w["query_known"]
    params = bm.bm_params_preset(2)
    ctx = bm.bm_ctx_create(params, 0)
    ks = [args.k] if args.k else [1, 2, 4, 8, 16]
    lm, ho = bm.BM_LEVEL_MIN, bm.BM_HOIST
    scheds = [args.schedule] if args.schedule else [1, 2, 1 | lm, 2 | lm, 2 | ho, 2 | lm | ho]
    rots = set()
    for k in ks:
        rots.update(bm.bm_rotations_for(d, k))
        rots.update(bm.bm_rotations_compress(d, k))
        if any(s & ho for s in scheds):
            rots.update(bm.bm_rotations_hoisted(d, k))
    t0 = time.time()
    sk, pk, evk = bm.bm_keygen(ctx, seed, sorted(rots))
    q_ct = bm.bm_encrypt_query(ctx, pk, q, seed, 1)
    gals = {k: bm.bm_encrypt_gallery(ctx, pk, X, k, seed, 1000) for k in ks}
    print("# setup %.1fs (keys for %d rotations, %d galleries)" % (time.time() - t0, len(rots), len(ks)),
          file=sys.stderr, flush=True)
    # a dedicated stream: the library's launches and the timing events share it
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    sptr = stream.cuda_stream

    def run_once(k, s):
        r = bm.bm_match(ctx, evk, q_ct, gals[k], None, schedule=s, out_limbs=0, stream=sptr)
        return r

    # matches are captured once per configuration as HIP graphs and replayed
    bm.bm_ctx_set_graphs(ctx, not args.eager)

    # ---- short sweep over (k, schedule)
    def sname(s):
        return "S%d%s%s%s" % (s & 0xff, "+levelmin" if s & bm.BM_LEVEL_MIN else "",
                              "+hoist" if s & bm.BM_HOIST else "", "+compress" if s & bm.BM_COMPRESS else "")

    sweep, conf = {}, {}
    for k in ks:
        for s in scheds:
            if k == 1 and (s & 0xff) == 2 and (s - 1) in scheds:
                continue          # identical work for a single part
            bm.bm_result_free(run_once(k, s))
            torch.cuda.synchronize()
            t = time.perf_counter()
            reps = 2
            for _ in range(reps):
                bm.bm_result_free(run_once(k, s))
            torch.cuda.synchronize()
            key = "k%d_%s" % (k, sname(s))
            sweep[key] = (time.perf_counter() - t) * 1e3 / reps
            conf[key] = (k, s)
            print("# sweep %s: %.2f ms/match" % (key, sweep[key]), file=sys.stderr, flush=True)
    best = min(sweep, key=sweep.get)
    bk, bs = conf[best]
    # the result-invariant knobs of the chosen configuration, by the autotuner
    if args.tuning:
        knobs = [int(v) for v in args.tuning.split(",")]
        bm.bm_ctx_set_tuning(ctx, *knobs)
        tuning = bm.bm_ctx_get_tuning(ctx)
        print("# fixed knobs %s" % tuning, file=sys.stderr, flush=True)
    else:
        _, tuning, tuned_ms = bm.bm_autotune_batch(ctx, evk, [q_ct], [gals[bk]], [bs])
        print("# autotuned knobs %s: %.3f ms/match" % (tuning, tuned_ms), file=sys.stderr, flush=True)
    canon = {key: v for key, v in sweep.items() if not conf[key][1] & (bm.BM_LEVEL_MIN | bm.BM_HOIST)}
    canon_best = min(canon, key=canon.get) if canon else None

    # ---- the same match with the compression method: one result ciphertext
    # per c groups instead of one per group (what the client downloads)
    compressed = None
    if not bs & bm.BM_COMPRESS and not args.no_extras:
        cs = bs | bm.BM_COMPRESS
        bm.bm_result_free(run_once(bk, cs))
        torch.cuda.synchronize()
        t = time.perf_counter()
        rs = [run_once(bk, cs) for _ in range(3)]
        torch.cuda.synchronize()
        cms = (time.perf_counter() - t) * 1e3 / 3
        r = rs.pop()
        for x in rs:
            bm.bm_result_free(x)
        n_ct, climbs, _ = bm.bm_result_info(r)
        csc = bm.bm_decrypt_scores(ctx, sk, r, n_tmpl)
        bm.bm_result_free(r)
        r = run_once(bk, bs)
        n_plain, plimbs, _ = bm.bm_result_info(r)
        bm.bm_result_free(r)
        cos0 = X.astype(np.float64) @ q.astype(np.float64)
        compressed = {"config": "k%d_%s" % (bk, sname(cs)), "ms_per_match": round(cms, 3),
                      "result_ciphertexts": n_ct, "result_bytes": n_ct * 2 * climbs * params.N * 8,
                      "uncompressed_ciphertexts": n_plain,
                      "uncompressed_bytes": n_plain * 2 * plimbs * params.N * 8,
                      "max_abs_err_vs_fp64_cosine": float(np.max(np.abs(csc - cos0)))}
        print("# compressed %s: %.2f ms/match, %d -> %d result ciphertexts" %
              (compressed["config"], cms, n_plain, n_ct), file=sys.stderr, flush=True)

    # ---- timed region: each step's result is released once the next step is
    # enqueued, as a server hands its results off, so the steps reuse the
    # result memory the pool holds (stream order keeps a released result's
    # memory untouched until the match writing it is done)
    prev = None
    for _ in range(args.warmup):
        r = run_once(bk, bs)
        if prev is not None:
            bm.bm_result_free(prev)
        prev = r
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        r = run_once(bk, bs)
        ends[i].record(stream)
        if prev is not None:
            bm.bm_result_free(prev)
        prev = r
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    lat = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    scores = bm.bm_decrypt_scores(ctx, sk, prev, n_tmpl)
    bm.bm_result_free(prev)

    # ---- the same match with host buffers on both sides (never `value`): the
    # query handed over from pinned host memory in the coefficient domain (the
    # import runs its forward NTT), every result ciphertext copied back (the
    # export runs the inverse NTT, one launch and one copy for all of them),
    # each call synchronous
    pcie = None
    if not args.no_extras:
        qwords, qscale = bm.bm_ct_export(ctx, q_ct, params.N)
        hq = torch.from_numpy(qwords.view(np.int64)).pin_memory()
        hq_np = hq.numpy().view(np.uint64)
        r0 = run_once(bk, bs)
        G, olimbs, _ = bm.bm_result_info(r0)
        bm.bm_result_free(r0)
        per = 2 * olimbs * params.N
        hout = torch.empty((G, per), dtype=torch.int64).pin_memory()
        L = bm.lib()

        def pcie_once():
            qc = bm.bm_ct_import(ctx, hq_np, qscale)
            r = bm.bm_match(ctx, evk, qc, gals[bk], None, schedule=bs, out_limbs=0, stream=sptr)
            st = L.bm_result_export_all(r, hout.data_ptr(), G * per)    # every result in one transfer
            if st != bm.BM_OK:
                raise bm.BMError(st, "bm_result_export_all", "")
            bm.bm_result_free(r)
            bm.bm_ct_free(qc)
        for _ in range(2):
            pcie_once()
        torch.cuda.synchronize()
        reps = 10
        t = time.perf_counter()
        for _ in range(reps):
            pcie_once()
        torch.cuda.synchronize()
        pms = (time.perf_counter() - t) * 1e3 / reps
        got = hout.numpy().view(np.uint64)
        r = run_once(bk, bs)
        same = all(np.array_equal(got[g].reshape(2, olimbs, params.N), bm.bm_result_export(ctx, r, g, params.N)[0])
                   for g in range(G))
        bm.bm_result_free(r)
        pcie = {"ms_per_match": round(pms, 3), "templates_per_s": round(n_tmpl / pms * 1e3, 1),
                "h2d_bytes": int(qwords.nbytes), "d2h_bytes": int(hout.numel() * 8),
                "host_memory": "pinned", "results_equal_resident_path": bool(same)}
        print("# host buffers (PCIe-inclusive): %.3f ms/match" % pms, file=sys.stderr, flush=True)

    # ---- per-kernel times: the same steps once more, launched eagerly with a
    # HIP event pair around every kernel on its stream (a graph replay cannot
    # be bracketed kernel by kernel)
    prof, eager_ms = {}, None
    if not args.no_profile:
        bm.bm_profile_enable(ctx, True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(args.steps):
            bm.bm_result_free(run_once(bk, bs))
        torch.cuda.synchronize()
        eager_ms = (time.perf_counter() - t1) * 1e3 / args.steps
        prof = bm.bm_profile_dump(ctx)
        bm.bm_profile_enable(ctx, False)
    cos = X.astype(np.float64) @ q.astype(np.float64)
    err = float(np.max(np.abs(scores - cos)))
    top = bm.bm_top1(scores)[0]
    ms_step = elapsed * 1e3 / args.steps
    value = n_tmpl * args.steps / elapsed

    # ---- roofline: every kernel on its own (HIP events stamped with each
    # launch's execution interval), the one with the most device time as the
    # headline entry, and the whole match against its compulsory traffic
    roof = None
    if prof:
        roof = roofline_entries(prof, args.steps)
        top = roof["kernels"][0]
        e = prof[top["kernel"]]
        roof["traffic"] = traffic_for(top["kernel"], "k%d_%s" % (bk, sname(bs)), top["algorithmic_bytes_per_launch"])
        # the same kind of arithmetic at its measured register-resident rate
        mrate = measured_butterfly_rate(bm, ctx, params)
        roof["alu_measured_peak_gmodmul"] = round(mrate, 1)
        roof["alu_frac_measured"] = round(roof["alu_gmodmul"] / mrate, 4)
        step_ms_dev = sum(v["ms"] for v in prof.values()) / args.steps
        roof["kernel_share"] = round(e["ms"] / args.steps / max(step_ms_dev, 1e-9), 3)
        mb = match_compulsory_bytes(params, d, bk, bm.bm_gallery_info(gals[bk])[0], bs, params.out_limbs, bm)
        roof["match"] = dict(compulsory_bytes=int(mb["total"]), parts=mb["parts"], ms_per_step=round(ms_step, 4),
                             achieved_gbs=round(mb["total"] / (ms_step * 1e-3) / 1e9, 1),
                             frac=round(mb["total"] / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                             device_ms_per_step_eager=round(step_ms_dev, 4))
        breakdown = {n: round(v["ms"] / args.steps, 3) for n, v in sorted(prof.items(), key=lambda x: -x[1]["ms"])}
    else:
        breakdown = {}

    # ---- the same workload in the conjugate-invariant ring (the paper's
    # setting: N real slots, so half the gallery ciphertexts)
    ci = None
    if not args.no_ci and not args.no_extras:
        ci_scheds = sorted({s for s in scheds if s & bm.BM_LEVEL_MIN} or {bs})
        ci = ci_variant(bm, torch, X, q, d, ks, ci_scheds, w["known"], sptr, not args.eager, sname)

    # ---- CPU oracle on a bounded sample (one gallery group, same k and schedule)
    cpu = cpu1 = None
    if not args.no_cpu:
        cpu = cpu_baseline(bk, bs, X, q, d)
        print("# cpu oracle (all threads): %s templates/s" % cpu["value"], file=sys.stderr, flush=True)
        if not args.no_extras:
            cpu1 = cpu_single_thread(bk, bs, d)
            print("# cpu oracle (one thread): %s templates/s" % (cpu1 or {}).get("value"),
                  file=sys.stderr, flush=True)

    # ---- the other workloads: fingerprint scale (C3), the mixed batch (C4)
    # and serving (C5), each a summary in config (their own lines with
    # --workload fingerprint | batch | serve)
    others = {}
    if not args.no_extras and not args.no_workloads:
        import bench_workloads
        for key, fn in (("fingerprint", bench_workloads.fingerprint), ("batched", bench_workloads.batch),
                        ("serving", bench_workloads.serve)):
            t_w = time.time()
            try:
                others[key] = fn(bm, args)
            except Exception as ex:         # reported, never fatal to the headline line
                others[key] = {"error": repr(ex)[:400]}
            print("# workload %s: %.1fs" % (key, time.time() - t_w), file=sys.stderr, flush=True)
        torch.cuda.set_stream(stream)

    out = {
        "metric": "encrypted templates scored/s (N=2^16, 128-dim); p50/p99 query latency",
        "value": round(value, 1),
        "unit": "templates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "face-scale 1:N match: N=2^16, 8x50-bit chain + 2x51-bit special primes, "
                        "dnum=4, 6144 x 128-dim templates in 24 ciphertexts, one query",
            "k": bk, "schedule": sname(bs), "tuning": tuning, "templates": n_tmpl, "compressed": compressed,
            "natural_level_best": ({"config": canon_best, "ms_per_match": round(canon[canon_best], 3),
                                    "templates_per_s": round(n_tmpl / canon[canon_best] * 1e3, 1)}
                                   if canon_best else None),
            "step_latency": {"p50_ms": round(float(np.percentile(lat, 50)), 3),
                             "p99_ms": round(float(np.percentile(lat, 99)), 3),
                             "what": "back-to-back graph replays of one match on one stream (HIP events per "
                                     "step); no arrivals or queueing: served query latency is config.serving"},
            "arithmetic": "exact integer residues mod primes below 2^51, held in HBM as 64-bit words; the "
                          "transforms, key inner products and tensor carry them as exact integers in FP64 "
                          "registers (the ALU figures are FP64 issue rates)",
            "sweep_ms": {k: round(v, 3) for k, v in sweep.items()},
            "max_abs_err_vs_fp64_cosine": err, "top1_correct": bool(top == w["known"]),
            "kernel_ms_per_step": breakdown,
            "launch": "eager" if args.eager else "hip_graph",
            "eager_profiled_ms_per_step": round(eager_ms, 3) if eager_ms else None,
            "conjugate_invariant_ring": ci,
            "host_buffers_pcie_inclusive": pcie,
            "cpu_oracle_single_thread": cpu1,
            "fingerprint": others.get("fingerprint"),
            "batched": others.get("batched"),
            "serving": others.get("serving"),
            "paper_context": "Lattigo CPU, N=8192 real slots, 3 clusters x 2 Xeon Gold 5220 cores: "
                             "6144 x 128-dim matched in 451.67 ms (13,603 templates/s)",
        },
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def roofline_entries(prof, steps):
    """The roofline of a profiled run: every kernel on its own (its algorithmic
    bytes per launch over its average duration, HIP events stamped with each
    launch's execution interval), the kernel with the most device time as the
    headline entry."""
    kernels = []
    for n, e in sorted(prof.items(), key=lambda x: -x[1]["ms"]):
        avg_s = e["ms"] / e["launches"] / 1e3
        bpl = e["bytes"] / e["launches"]
        kernels.append(dict(kernel=n, launches_per_step=round(e["launches"] / steps, 2),
                            avg_us=round(avg_s * 1e6, 2), algorithmic_bytes_per_launch=int(bpl),
                            achieved_gbs=round(bpl / avg_s / 1e9, 1),
                            frac=round(bpl / avg_s / 1e9 / HBM_PEAK_GBS, 4),
                            ms_per_step=round(e["ms"] / steps, 4)))
    top = kernels[0]
    e = prof[top["kernel"]]
    avg_s = e["ms"] / e["launches"] / 1e3
    gmm = e["ops"] / e["launches"] / avg_s / 1e9
    return dict(bound="hbm", kernel=top["kernel"], achieved=top["achieved_gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                frac=top["frac"], avg_us=top["avg_us"], launches_per_step=top["launches_per_step"],
                algorithmic_bytes_per_launch=top["algorithmic_bytes_per_launch"],
                alu_gmodmul=round(gmm, 2), alu_frac=round(gmm / ALU_PEAK_GMODMUL, 4), traffic=None,
                kernels=kernels)


def match_compulsory_bytes(p, d, k, G, schedule, ctx_out_limbs, bm):
    """Bytes one match must move at least: every gallery word at the limbs the
    products use, every key word the key switches read (each key once, over
    the target slots of its level), the query and the masks once, the result
    ciphertexts once.  Mirrors the library's plan of the match (levels of
    the products, of the rotate-and-sum and of the output).  No compression."""
    N, L1, K, alpha = p.N, p.n_q, p.n_p, p.alpha
    lmin, hoist = bool(schedule & bm.BM_LEVEL_MIN), bool(schedule & bm.BM_HOIST)
    g_limbs = L1 if k == 1 else L1 - 1
    t = min(3, g_limbs) if lmin else g_limbs
    ql = t + 1 if k > 1 else t
    nat = t - 1
    ol = min(ctx_out_limbs or nat, nat)
    rot = ol if lmin else nat
    c = d // k

    def key_words(limbs):        # one switching key read over the target slots of `limbs`
        beta = -(-limbs // alpha)
        return 2 * beta * (limbs + K) * N

    if k > 1:
        if hoist:
            amounts = set()
            for i in range(k):
                for S in range(1, k):
                    r = 0
                    for tt in range(k.bit_length() - 1):
                        if (S >> tt) & 1:
                            r += (c << tt) if (i >> tt) & 1 else -(c << tt)
                    amounts.add(r)
            n_exp = len(amounts)
        else:
            n_exp = 2 * (k.bit_length() - 1)
    else:
        n_exp = 0
    n_rot = (c - 1) if hoist else (c.bit_length() - 1)
    parts = {
        "gallery": 8 * G * k * 2 * t * N,
        "query": 8 * 2 * ql * N,
        "masks": 8 * k * ql * N if k > 1 else 0,
        "expansion_keys": 8 * n_exp * key_words(ql - 1),
        "relinearisation_key": 8 * key_words(t),
        "rotation_keys": 8 * n_rot * key_words(rot),
        "results": 8 * G * 2 * ol * N,
    }
    return {"total": sum(parts.values()), "parts": parts}


def ci_variant(bm, torch, X, q, d, ks, scheds, known, sptr, graphs, sname, reps=10):
    """The face-scale match over the conjugate-invariant ring of the same rank
    (preset 4: N = 2^16 real slots, so twice the templates per ciphertext),
    library encryption; short sweep over the given k and schedules, then the
    best timed over `reps` matches."""
    params = bm.bm_params_preset(4)
    ctx = bm.bm_ctx_create(params, 0)
    rots = set()
    for k in ks:
        rots.update(bm.bm_rotations_for(d, k))
        if any(s & bm.BM_HOIST for s in scheds):
            rots.update(bm.bm_rotations_hoisted(d, k))
    sk, pk, evk = bm.bm_keygen(ctx, 0xC1, sorted(rots))
    q_ct = bm.bm_encrypt_query(ctx, pk, q, 0xC1, 1)
    gals = {k: bm.bm_encrypt_gallery(ctx, pk, X, k, 0xC1, 1000) for k in ks}
    bm.bm_ctx_set_graphs(ctx, graphs)

    def once(k, s):
        return bm.bm_match(ctx, evk, q_ct, gals[k], None, schedule=s, out_limbs=0, stream=sptr)

    def timed(k, s, n):
        bm.bm_result_free(once(k, s))
        torch.cuda.synchronize()
        t = time.perf_counter()
        rs = [once(k, s) for _ in range(n)]
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / n, rs

    sweep = {}
    for k in ks:
        for s in scheds:
            ms, rs = timed(k, s, 2)
            for r in rs:
                bm.bm_result_free(r)
            sweep[(k, s)] = ms
    k, s = min(sweep, key=sweep.get)
    ms, rs = timed(k, s, reps)
    scores = bm.bm_decrypt_scores(ctx, sk, rs[-1], X.shape[0])
    for r in rs:
        bm.bm_result_free(r)
    cos = X.astype(np.float64) @ q.astype(np.float64)
    groups = bm.bm_gallery_info(gals[k])[0]
    out = {"ring": "Z[X+X^-1], N=2^16 real slots (primes 1 mod 4N)", "k": k, "schedule": sname(s),
           "gallery_groups": groups, "ms_per_match": round(ms, 3),
           "templates_per_s": round(X.shape[0] / ms * 1e3, 1),
           "max_abs_err_vs_fp64_cosine": float(np.max(np.abs(scores - cos))),
           "top1_correct": bool(bm.bm_top1(scores)[0] == known),
           "sweep_ms": {"k%d_%s" % (kk, sname(ss)): round(v, 3) for (kk, ss), v in sweep.items()}}
    print("# conjugate-invariant ring: k=%d %s, %d groups, %.3f ms/match" % (k, sname(s), groups, ms),
          file=sys.stderr, flush=True)
    bm.bm_ct_free(q_ct)
    for g in gals.values():
        bm.bm_gallery_free(g)
    bm.bm_sk_free(sk)
    bm.bm_pk_free(pk)
    bm.bm_evk_free(evk)
    bm.bm_ctx_free(ctx)
    return out


def cpu_baseline(k, schedule, X, q, d, budget_s=10.0, max_groups=None):
    """The oracle as it stands on the same workload and schedule, group after
    group until about `budget_s` of CPU time is spent (expansion counted once,
    as in one query), scaled to templates/s."""
    from oracle import ckks, blindmatch as obm
    P = ckks.Params.preset(2)
    c, T = obm.layout(P, d, k)
    lmin, hoist, sch = bool(schedule & 0x100), bool(schedule & 0x400), schedule & 0xff
    rots = set(obm.rotations_needed(P, d, k))
    if hoist:
        rots.update(obm.hoisted_rotations(P, d, k))
    keys = ckks.keygen(P, 0xB11D, sorted(rots))
    m = ckks.encode(obm.pack_query(P, q.astype(np.float64), d), P.scale, P.N)
    cq = ckks.encrypt(P, keys.pk, m, len(P.q), P.scale, 0xB11D, 1)
    lg = obm.gallery_limbs(P, k)
    groups = obm.pack_gallery(P, X.astype(np.float64), d, k)
    t_l, ql = obm.level_min_shape(P, k, lg) if lmin else (lg, len(P.q))
    masks, mscale = obm.mask_coeffs(P, d, k, ql) if k > 1 else (None, None)
    t0 = time.perf_counter()
    cq_used = ckks.drop_limbs(cq, ql) if lmin else cq
    if k == 1:
        cu = [cq_used]
    else:
        cu = (obm.expand_hoisted if hoist else obm.expand)(P, keys, cq_used, d, k, masks, mscale)
    dt = time.perf_counter() - t0          # matching time only; gallery encryption is setup
    done = 0
    for g, part_slots in enumerate(groups):
        gal = [ckks.encrypt(P, keys.pk, ckks.encode(v, P.scale, P.N), lg, P.scale, 0xB11D, 1000 + g * k + i)
               for i, v in enumerate(part_slots)]
        t1 = time.perf_counter()
        if lmin:
            gal = [ckks.drop_limbs(x, t_l) for x in gal]
        out = obm.hec3(P, keys, cu, gal, d, k, sch, rot_limbs=2 if lmin else None, hoist=hoist)
        ckks.drop_limbs(out, 2)
        dt += time.perf_counter() - t1
        done += min(T, X.shape[0] - g * T)
        if dt >= budget_s or (max_groups and g + 1 >= max_groups):
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=round(done / dt, 1), unit="templates/s", cores=cores, kind="oracle",
                sample="%d of %d templates (%d of %d groups, k=%d, schedule %#x%s), %.1fs of oracle time"
                       % (done, X.shape[0], g + 1, len(groups), k, schedule, ", one expansion" if k > 1 else "", dt))


def measured_butterfly_rate(bm, ctx, params, blocks=2048, iters=4096):
    """G butterflies/s of the library's register-resident probe (8 independent
    FP64 butterfly chains per thread, folded every second round as in the NTT)
    on the first chain prime: the ALU ceiling actually reachable with this
    arithmetic, beside the one derived from unit counts."""
    q = params.chain()[0]
    seed = np.random.default_rng(0x5EED).integers(0, q, size=24, dtype=np.uint64)
    bm.bm_bench_modmul(ctx, 0, blocks, 64, seed)          # warm-up
    ms = min(bm.bm_bench_modmul(ctx, 0, blocks, iters, seed)[0] for _ in range(3))
    return blocks * 256 * 8 * iters / (ms * 1e-3) / 1e9


def cpu_single_thread(k, schedule, d):
    """The oracle sample on one host thread: a child process, because OpenMP
    takes its thread count when the oracle's library is loaded."""
    import subprocess
    code = ("import json, sys; sys.path.insert(0, %r); import bench; from workloads import face_gallery; "
            "w = face_gallery(seed=2, d=%d, n=6144); "
            "print(json.dumps(bench.cpu_baseline(%d, %d, w['gallery'], w['query_known'], %d, budget_s=1.0)))"
            % (ROOT, d, k, schedule, d))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=900)
    except subprocess.TimeoutExpired:
        return None
    if r.returncode != 0:
        print("# single-thread oracle failed: " + r.stderr[-500:], file=sys.stderr, flush=True)
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


if __name__ == "__main__":
    main()
