"""Secondary benchmarks of bench.py (--workload fingerprint | batch | serve).

fingerprint: one query against 1,048,576 L2-normalised 16-dim templates from a
             clustered Gaussian mixture (1,000 identities), k = 1, 512
             ciphertexts at N = 2^16: the large-gallery streaming case.
batch:       64 queries of dimension 16, 64, 128, 512 (16 each) against two
             galleries of uneven size per dimension (128 pairs), matched
             (a) pair by pair with the plain path and (b) with bm_match_batch,
             which batches all queries of a gallery into each launch.
copy:        a plain device-to-device copy of 1 GiB, timed: the HBM bandwidth a
             copy reaches, and the known-size dispatch that scales the
             FETCH_SIZE / WRITE_SIZE counters of the other kernels to bytes.
serve:       the continuous-batching server over 16 resident galleries (twelve
             128-dim, four 16-dim), Poisson arrivals at several rates, a 3:1
             mix of 128-dim to 16-dim queries; p50/p99 latency and admitted
             throughput, against the plain per-query path.
Each prints one JSON line.  --scale shrinks the batch/serve galleries.
"""
import json
import sys
import time

import numpy as np


def _setup(bm, shapes, seed=0xB11D):
    import torch
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    ctx = bm.bm_ctx_create(bm.bm_params_preset(2), 0)
    rots = set()
    for d, k in shapes:
        rots.update(bm.bm_rotations_for(d, k))
    sk, pk, evk = bm.bm_keygen(ctx, seed, sorted(rots))
    return torch, stream, ctx, sk, pk, evk


def run(args):
    import paper_2408_06167_amd as bm
    {"fingerprint": fingerprint, "batch": batch, "serve": serve, "copy": copy, "ntt": ntt}[args.workload](bm, args)


def fingerprint(bm, args):
    from workloads import fingerprint_gallery
    d, k, seed = 16, 1, 0xB11D
    w = fingerprint_gallery(seed=3, d=d, n=1 << 20)
    X, q = w["gallery"], w["query"]
    torch, stream, ctx, sk, pk, evk = _setup(bm, [(d, k)])
    t0 = time.time()
    gal = bm.bm_encrypt_gallery(ctx, pk, X, k, seed, 1 << 20)
    cq = bm.bm_encrypt_query(ctx, pk, q, seed, 1)
    G, _, _ = bm.bm_gallery_info(gal)
    print("# gallery of %d ciphertexts encrypted in %.1fs" % (G, time.time() - t0), file=sys.stderr, flush=True)
    bm.bm_ctx_set_graphs(ctx, True)
    out = {}
    for name, sched in (("S1", 1), ("S1+levelmin", 1 | bm.BM_LEVEL_MIN)):
        chunk, ms_tuned = bm.bm_autotune(ctx, evk, cq, gal, sched)
        bm.bm_result_free(bm.bm_match(ctx, evk, cq, gal, None, schedule=sched, stream=stream.cuda_stream))
        torch.cuda.synchronize()
        lat = []
        for _ in range(max(3, args.steps // 4)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            r = bm.bm_match(ctx, evk, cq, gal, None, schedule=sched, stream=stream.cuda_stream)
            e1.record(stream)
            torch.cuda.synchronize()
            lat.append(e0.elapsed_time(e1))
            last = r if len(lat) == 1 else (bm.bm_result_free(r) or last)
        scores = bm.bm_decrypt_scores(ctx, sk, last, X.shape[0])
        bm.bm_result_free(last)
        cos = X.astype(np.float64) @ q.astype(np.float64)
        err = float(np.max(np.abs(scores - cos)))
        ms = float(np.median(lat))
        out[name] = dict(ms_per_query=round(ms, 3), templates_per_s=round(X.shape[0] / ms * 1e3, 1),
                         group_chunk=chunk, max_abs_err=err,
                         top1_identity_ok=bool(int(bm.bm_top1(scores)[0]) % w["identities"] == w["query_identity"]))
        print("# %s: %.2f ms/query (chunk %d), err %.1e" % (name, ms, chunk, err), file=sys.stderr, flush=True)
    best = min(out, key=lambda n: out[n]["ms_per_query"])
    cpu = None
    if not args.no_cpu:            # the oracle on a bounded sample of the same gallery and schedule
        import bench
        cpu = bench.cpu_baseline(k, 1 | (bm.BM_LEVEL_MIN if "levelmin" in best else 0), X, q, d, budget_s=10.0)
        print("# cpu oracle: %s templates/s (%s)" % (cpu["value"], cpu["sample"]), file=sys.stderr, flush=True)
    print(json.dumps({"metric": "encrypted templates scored/s (N=2^16, 16-dim, 1,048,576 templates)",
                      "value": out[best]["templates_per_s"], "unit": "templates/s", "n_gpus": 1,
                      "higher_is_better": True, "data": "synthetic", "dtype": "u64",
                      "config": {"workload": "fingerprint-scale: 1,048,576 x 16-dim, k=1, %d ciphertexts" % G,
                                 "schedule": best, "variants": out},
                      "cpu_baseline": cpu}), flush=True)


def batch(bm, args):
    from workloads import mixed_batch
    wl = mixed_batch(seed=4, scale_sizes=args.scale)
    kfor = {16: 1, 64: 2, 128: 4, 512: 16}          # chunk c = d/k = 16 or 32
    shapes = sorted({(g["d"], kfor[g["d"]]) for g in wl["galleries"]})
    torch, stream, ctx, sk, pk, evk = _setup(bm, shapes)
    sched = 2 | bm.BM_LEVEL_MIN
    t0 = time.time()
    gals = [bm.bm_encrypt_gallery(ctx, pk, g["X"], kfor[g["d"]], 0xB11D, 100000 * i)
            for i, g in enumerate(wl["galleries"])]
    qs = [bm.bm_encrypt_query(ctx, pk, qd["q"], 0xB11D, 10 + i) for i, qd in enumerate(wl["queries"])]
    pairs = [(qi, gi) for qi, qd in enumerate(wl["queries"])
             for gi, g in enumerate(wl["galleries"]) if g["d"] == qd["d"]]
    n_templates = sum(wl["galleries"][gi]["X"].shape[0] for _, gi in pairs)
    print("# %d pairs, %d templates scored, setup %.1fs" % (len(pairs), n_templates, time.time() - t0),
          file=sys.stderr, flush=True)
    bm.bm_ctx_set_graphs(ctx, True)

    def plain():
        outs = []
        for qi, gi in pairs:
            outs.append(bm.bm_match(ctx, evk, qs[qi], gals[gi], None, schedule=sched, stream=stream.cuda_stream))
        return outs

    def batched():
        return bm.bm_match_batch(ctx, evk, [qs[qi] for qi, _ in pairs], [gals[gi] for _, gi in pairs],
                                 schedule=sched, stream=stream.cuda_stream)

    res = {}
    keep = {}
    for name, fn in (("plain_per_pair", plain), ("batched", batched)):
        for r in fn():                                   # warm-up (graph capture, pools)
            bm.bm_result_free(r)
        torch.cuda.synchronize()
        t = time.perf_counter()
        outs = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        res[name] = dict(seconds=round(dt, 4), templates_per_s=round(n_templates / dt, 1))
        keep[name] = outs
        print("# %s: %.3fs" % (name, dt), file=sys.stderr, flush=True)
    # the two forms agree word for word (sampled pairs, first and last group)
    same = True
    for i in (0, len(pairs) // 2, len(pairs) - 1):
        a, b = keep["plain_per_pair"][i], keep["batched"][i]
        G, _, _ = bm.bm_result_info(a)
        for g in (0, G - 1):
            same &= bool(np.array_equal(bm.bm_result_export(ctx, a, g, 1 << 16)[0],
                                        bm.bm_result_export(ctx, b, g, 1 << 16)[0]))
    for outs in keep.values():
        for r in outs:
            bm.bm_result_free(r)
    print(json.dumps({"metric": "encrypted templates scored/s, mixed batch (N=2^16)",
                      "value": res["batched"]["templates_per_s"], "unit": "templates/s", "n_gpus": 1,
                      "higher_is_better": True, "data": "synthetic", "dtype": "u64",
                      "config": {"workload": "64 queries (d=16,64,128,512) x 2 galleries each, sizes x%.3g"
                                 % args.scale, "pairs": len(pairs), "templates": n_templates,
                                 "schedule": "S2+levelmin", "k_by_d": kfor, "results": res,
                                 "speedup_batched_over_plain": round(res["plain_per_pair"]["seconds"]
                                                                     / res["batched"]["seconds"], 3),
                                 "batched_equals_plain_sampled": same}}), flush=True)


def serve(bm, args):
    from workloads import serving_galleries, poisson_arrivals, normalize
    gl = serving_galleries(seed=5, scale_sizes=args.scale)
    kfor = {16: 1, 128: 4}
    torch, stream, ctx, sk, pk, evk = _setup(bm, [(16, 1), (128, 4)])
    sched = 2 | bm.BM_LEVEL_MIN
    t0 = time.time()
    srv = bm.bm_server_create(ctx, evk, 64 << 30, sched)
    by_d = {16: [], 128: []}
    sizes = {}
    plain_gals = {}
    for i, g in enumerate(gl):
        h = bm.bm_encrypt_gallery(ctx, pk, g["X"], kfor[g["d"]], 0xB11D, 1000000 * (i + 1))
        gid = bm.bm_server_add_gallery(srv, h)
        by_d[g["d"]].append(gid)
        sizes[gid] = g["X"].shape[0]
        if i in (0, len(gl) - 4):                        # one gallery per dimension for the plain path
            plain_gals[g["d"]] = (bm.bm_encrypt_gallery(ctx, pk, g["X"], kfor[g["d"]], 0xB11D,
                                                        1000000 * (i + 1)), g["X"].shape[0])
    print("# %d galleries, %d templates, setup %.1fs" % (len(gl), sum(sizes.values()), time.time() - t0),
          file=sys.stderr, flush=True)
    rng = np.random.default_rng(55)
    out = {}
    for rate in [float(r) for r in args.rates.split(",")]:
        t_arr, dims, picks = poisson_arrivals(int(rate * 1000), rate, args.requests)
        # clients encrypt ahead of time; the server sees ciphertexts arrive
        cts = [bm.bm_encrypt_query(ctx, pk, normalize(rng.standard_normal(int(dd))), 0xB11D, 50000 + i)
               for i, dd in enumerate(dims)]
        routes = [by_d[int(dd)][int(p) % len(by_d[int(dd)])] for dd, p in zip(dims, picks)]
        bm.bm_server_reset_stats(srv)
        start = time.perf_counter()
        tickets = []
        for i in range(len(cts)):
            now = time.perf_counter() - start
            if t_arr[i] > now:
                time.sleep(t_arr[i] - now)
            tickets.append(bm.bm_server_submit(srv, routes[i], cts[i]))
        bm.bm_server_drain(srv)
        wall = time.perf_counter() - start
        scored = 0
        for tk, gid in zip(tickets, routes):
            r = bm.bm_server_poll(srv, tk)
            scored += sizes[gid]
            bm.bm_result_free(r)
        st = bm.bm_server_stats(srv)
        out["%g" % rate] = dict(p50_ms=round(st["p50_ms"], 2), p99_ms=round(st["p99_ms"], 2),
                                mean_batch=round(st["mean_batch"], 2),
                                templates_per_s=round(scored / wall, 1), queries_per_s=round(len(cts) / wall, 2))
        print("# rate %g: %s" % (rate, out["%g" % rate]), file=sys.stderr, flush=True)
        bm.bm_server_reset_stats(srv)
    # plain per-query path on the same shapes for comparison
    bm.bm_ctx_set_graphs(ctx, True)
    plain = {}
    for dd, (h, n) in plain_gals.items():
        q = bm.bm_encrypt_query(ctx, pk, normalize(rng.standard_normal(dd)), 0xB11D, 9)
        bm.bm_result_free(bm.bm_match(ctx, evk, q, h, None, schedule=sched, stream=stream.cuda_stream))
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(5):
            bm.bm_result_free(bm.bm_match(ctx, evk, q, h, None, schedule=sched, stream=stream.cuda_stream))
        torch.cuda.synchronize()
        plain["d%d_%d_templates" % (dd, n)] = round((time.perf_counter() - t) / 5 * 1e3, 3)
        bm.bm_ct_free(q)
    bm.bm_server_free(srv)
    best = max(out, key=lambda r: out[r]["templates_per_s"])
    print(json.dumps({"metric": "served encrypted templates/s with p50/p99 latency (N=2^16)",
                      "value": out[best]["templates_per_s"], "unit": "templates/s", "n_gpus": 1,
                      "higher_is_better": True, "data": "synthetic", "dtype": "u64",
                      "config": {"workload": "16 resident galleries (12 x 128-dim, 4 x 16-dim), sizes x%.3g, "
                                 "Poisson arrivals, 3:1 mix" % args.scale, "templates": sum(sizes.values()),
                                 "schedule": "S2+levelmin", "by_rate": out,
                                 "plain_ms_per_query": plain}}), flush=True)


def ntt(bm, args):
    """Batched negacyclic NTT at N = 2^16 through bm_ntt, in place on device
    words[polys][8][N] (the 8 chain primes), forward and inverse, small and
    large batches, both rings.  Each transform is two passes that each read
    and write every word once: 32 bytes per word of algorithmic traffic."""
    import torch
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    rows = []
    for preset in (2, 4):
        p = bm.bm_params_preset(preset)
        ctx = bm.bm_ctx_create(p, 0)
        N, L1 = p.N, p.n_q
        ids = list(range(L1))
        for polys in (1, 4, 32):
            rng = np.random.default_rng(polys)
            host = np.stack([np.stack([rng.integers(0, q, N, dtype=np.uint64) for q in p.chain()])
                             for _ in range(polys)])
            dev = torch.from_numpy(host.view(np.int64).copy()).cuda()
            for inv in (False, True):
                bm.bm_ntt(ctx, dev.data_ptr(), polys, ids, inv, stream.cuda_stream)
            torch.cuda.synchronize()
            for inv in (False, True):
                reps = max(args.steps, 5)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(reps):
                    bm.bm_ntt(ctx, dev.data_ptr(), polys, ids, inv, stream.cuda_stream)
                e1.record(stream)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                words = polys * L1 * N
                bfly = words // 2 * 16
                rows.append(dict(ring="conjugate-invariant" if preset == 4 else "standard", limb_polys=polys * L1,
                                 direction="inverse" if inv else "forward", us=round(ms * 1e3, 2),
                                 gb_s=round(32.0 * words / ms / 1e6, 1), gbfly_s=round(bfly / ms / 1e6, 1)))
                print("# %s %s, %d limb-polynomials: %.1f us, %.0f GB/s" % (
                    rows[-1]["ring"], rows[-1]["direction"], polys * L1, ms * 1e3, rows[-1]["gb_s"]),
                    file=sys.stderr, flush=True)
            # the round trip gives back the input words (in the conjugate-invariant
            # ring only for invariant inputs, which random words are not)
            if preset == 2:
                assert np.array_equal(dev.cpu().numpy().view(np.uint64), host)
            del dev
        bm.bm_ctx_free(ctx)
    big = [r for r in rows if r["limb_polys"] == 256 and r["ring"] == "standard"]
    print(json.dumps({"metric": "batched negacyclic NTT throughput (N=2^16, in place, 2 passes)",
                      "value": round(min(r["gb_s"] for r in big), 1), "unit": "GB/s", "n_gpus": 1,
                      "higher_is_better": True, "data": "synthetic", "dtype": "u64",
                      "config": {"workload": "bm_ntt on words[polys][8][65536], standard and conjugate-invariant rings",
                                 "rows": rows}}), flush=True)


def copy(bm, args):
    """1 GiB device copy: read 1 GiB, write 1 GiB per dispatch."""
    import torch
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    nbytes = 1 << 30
    src = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(max(args.warmup, 1)):
        dst.copy_(src)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for a, b in ev:
        a.record(stream)
        dst.copy_(src)
        b.record(stream)
    torch.cuda.synchronize()
    ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
    assert bool((dst[:: 1 << 20] == 1).all())
    print(json.dumps({"metric": "device copy bandwidth (read + write)", "value": round(2 * nbytes / ms / 1e6, 1),
                      "unit": "GB/s", "bytes_read_per_dispatch": nbytes, "bytes_written_per_dispatch": nbytes,
                      "ms_median": round(ms, 4), "dispatches": args.steps}))
