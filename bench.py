"""Throughput benchmark of the LCP hot path on one MI355X.

Default workload (the headline value): the MD-like trajectory, 64 frames of
4,194,304 particles on a 256x128x128 jittered lattice (spacing 1.0, jitter sigma
0.1, per-step Gaussian displacement sigma 0.01), float32 xyz, eb = 1e-4 x value
range of the first frame, Alg. 1 batches of 16 frames with LCP-FSM choosing S
or T per frame.  One step = compress the 64 frames (one multi-frame stream) +
decompress them (a second plan replays the stream).  The inputs are resident in
HBM before the timed region.  Throughput follows Eq. 4: size(D) / time,
size(D) = 4 * F * n bytes per frame.

Further legs (extra keys of the one JSON line): the uniform frame (2^18
particles, eb 1e-3, LCP-S only), the cosmology-like snapshot (2^27 particles x 6
fields, eb 1e-4 x range per field, LCP-S only), the batched form (256
independent frames per call) and the served form (32 streams).  Each leg reports
its whole-path fraction of the HBM roofline in algorithmic bytes:
  S compress 4FN + C, S decompress C + 4FN,
  T compress 4FN (frame) + 4FN (reference codes) + 4N (permutation) + C + 4FN
  (new reference codes), T decompress C + 4FN + 4FN + 4FN.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "compress/decompress GB/s at fixed eb + ratio; batched/served vs plain, p99"
HBM_PEAK_GBPS = 8000.0

# The roofline is quoted on the dominant kernel of the headline step, the
# temporal residual kernel; its algorithmic bytes per particle are its share of
# LCP-T compression's: the frame (12 B), the reference codes (12 B) and the slot
# permutation (4 B) read, the new reference codes (12 B) written.
ROOFLINE_KERNEL = "t_resid_run"

MALL_NOTE = ("the 256 MB Infinity Cache (MALL) holds a 4,194,304-particle frame's reference "
             "codes (48 MiB) and permutation (16 MiB), written by the previous launch, so part "
             "of this 'HBM' traffic is served from it")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def s_bytes(F, n, c):
    """Algorithmic bytes of one spatial frame (compress = decompress = 4FN + C)."""
    return 4 * F * n + c


def t_bytes_c(F, n, c):
    return 12 * F * n + 4 * n + c


def t_bytes_d(F, n, c):
    return 12 * F * n + c


def path_frac(byts, seconds):
    gbps = byts / seconds / 1e9
    return {"algorithmic_bytes": int(byts), "seconds": seconds, "achieved_GBps": gbps,
            "peak_GBps": HBM_PEAK_GBPS, "frac": gbps / HBM_PEAK_GBPS}


def copy_ceiling(torch, dev, mib=2048, reps=5):
    """What a plain device copy and a plain read sustain on this GPU: torch's copy
    kernel over `mib` MiB (read + write counted) and a sum over the same buffer
    (read only), best of `reps`, timed with events on the current stream."""
    src = torch.ones(mib << 18, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    nbytes = src.numel() * 4
    best_c = best_r = 1e9
    for _ in range(reps):
        a, b, c = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        a.record()
        dst.copy_(src)
        b.record()
        src.sum()
        c.record()
        c.synchronize()
        best_c = min(best_c, a.elapsed_time(b) * 1e-3)
        best_r = min(best_r, b.elapsed_time(c) * 1e-3)
    del src, dst
    torch.cuda.empty_cache()
    return {"copy_GBps": 2 * nbytes / best_c / 1e9, "read_GBps": nbytes / best_r / 1e9,
            "buffer_MiB": mib, "how": "torch copy_ and sum over a device buffer, best of %d" % reps}


def cpu_model() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:  # noqa: BLE001
        pass
    return platform.processor()


def cpu_baseline(frames_np, eb_rel, batch, k, gpu_methods, n_bytes_frame):
    """The CPU oracle (one thread) on the first frames of the workload, timed per
    spatial and per temporal frame, then weighted by the methods the GPU stream
    used on all its frames, so that the figure has the same S/T mix."""
    import oracle as O
    st = O.Stream(O.EB_REL_GLOBAL, eb_rel, batch_size=batch, block_log2=k,
                  max_n=frames_np[0].shape[1])
    dec = O.Stream(O.EB_REL_GLOBAL, eb_rel, batch_size=batch, block_log2=k,
                   max_n=frames_np[0].shape[1])
    tc = {O.METHOD_S: [], O.METHOD_T: []}
    td = {O.METHOD_S: [], O.METHOD_T: []}
    for x in frames_np:
        t0 = time.perf_counter()
        rec, used, _ = st.compress(x)
        t1 = time.perf_counter()
        dec.decompress(rec)
        t2 = time.perf_counter()
        tc[used].append(t1 - t0)
        td[used].append(t2 - t1)
    mean = lambda v: sum(v) / len(v) if v else None  # noqa: E731
    n_s = sum(1 for m in gpu_methods if m == O.METHOD_S)
    n_t = len(gpu_methods) - n_s
    cs, ct, ds, dt = mean(tc[O.METHOD_S]), mean(tc[O.METHOD_T]), mean(td[O.METHOD_S]), mean(td[O.METHOD_T])
    if ct is None:  # no temporal frame in the sample: charge them as spatial ones
        ct, dt = cs, ds
    tot_c = n_s * cs + n_t * ct
    tot_d = n_s * ds + n_t * dt
    total = n_bytes_frame * len(gpu_methods)
    return dict(value=total / (tot_c + tot_d) / 1e9, unit="GB/s", cores=1, kind="oracle",
                sample=f"first {len(frames_np)} frames of the workload at full n "
                       f"({len(tc[O.METHOD_S])} spatial, {len(tc[O.METHOD_T])} temporal), per-frame "
                       f"compress+decompress times weighted by the GPU stream's mix ({n_s} spatial, "
                       f"{n_t} temporal of {len(gpu_methods)}): compress {total / tot_c / 1e9:.4f} "
                       f"GB/s, decompress {total / tot_d / 1e9:.4f} GB/s; spatial frame "
                       f"{cs:.2f}+{ds:.2f} s, temporal frame {ct:.2f}+{dt:.2f} s; host CPU: "
                       f"{cpu_model()}, nproc {os.cpu_count()}")


def bench_single_s(args, torch, lcp, name, x, eb_mode, eb, steps, warmup, timer, cpu_n):
    """One frame, LCP-S only (single-frame plan, block size searched on the frame):
    compress and decompress timed separately over `steps` calls."""
    dev = x.device
    F, n = x.shape
    size_d = 4 * F * n
    plan = lcp.Plan(eb, eb_mode, n_fields=F, block_log2=-1, sample=x, max_particles=n)
    k = plan.block_log2
    out = torch.empty(plan.bound(n) + 16, dtype=torch.uint8, device=dev)
    dec = torch.empty((F, n), dtype=torch.float32, device=dev)
    offs = None
    for _ in range(warmup):
        _, offs, _, _ = plan.compress([x], out=out)
        plan.decompress(out, offs, outs=[dec])
    torch.cuda.synchronize()
    plan.timer_set(timer)
    tc = td = 0.0
    for _ in range(steps):
        t0 = time.perf_counter()
        _, offs, _, _ = plan.compress([x], out=out)
        t1 = time.perf_counter()
        plan.decompress(out, offs, outs=[dec])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        tc += t1 - t0
        td += t2 - t1
    kms, kl, kb = plan.timer_read()
    c = offs[1]
    # error bound, every value, against the slot permutation
    _, offs2, _, perms = plan.compress([x], out=out, want_perm=True)
    assert offs2[1] == c
    plan.decompress(out, offs2, outs=[dec])
    perm = perms[0].long()
    lo = x.amin(dim=1).double()
    hi = x.amax(dim=1).double()
    worst = 0.0
    for f in range(F):
        e = (dec[f].double() - x[f][perm].double()).abs().max().item()
        ebf = eb if eb_mode == lcp.EB_ABS else eb * (hi[f] - lo[f]).item() if eb_mode == lcp.EB_REL_PER_FIELD \
            else eb * (hi.max() - lo.min()).item()
        assert e <= ebf, (name, f, e, ebf)
        worst = max(worst, e / ebf)
    res = {
        "workload": name, "particles": n, "fields": F, "block_log2": k,
        "compress_GBps": size_d * steps / tc / 1e9, "decompress_GBps": size_d * steps / td / 1e9,
        "GBps": size_d * steps / (tc + td) / 1e9, "ratio": size_d / c, "bits_per_value": 32.0 * c / size_d,
        "max_err_over_eb": worst, "steps": steps,
        "path_roofline": {"bound": "hbm", "compress": path_frac(s_bytes(F, n, c) * steps, tc),
                          "decompress": path_frac(s_bytes(F, n, c) * steps, td),
                          "bytes_rule": "S compress 4FN + C, S decompress C + 4FN"},
        "kernel_timer": {"kernel": timer, "launches": kl,
                         "avg_launch_us": kms / kl * 1e3 if kl else None,
                         "declared_bytes_per_launch": kb / kl if kl else None},
    }
    if n * 4 * F <= (256 << 20):
        res["mall_note"] = "the whole frame fits in the 256 MB Infinity Cache: cache- and launch-bound, not HBM-bound"
    if cpu_n:
        # the oracle on the first cpu_n particles of the same frame
        import oracle as O
        xs = x[:, :cpu_n].cpu().numpy()
        grids = O.grids_for(xs, {lcp.EB_ABS: O.EB_ABS, lcp.EB_REL_GLOBAL: O.EB_REL_GLOBAL,
                                 lcp.EB_REL_PER_FIELD: O.EB_REL_PER_FIELD}[eb_mode], eb)
        t0 = time.perf_counter()
        rec, _, _ = O.compress_s(xs, grids, k)
        t1 = time.perf_counter()
        O.decompress(rec)
        t2 = time.perf_counter()
        nb = 4 * F * cpu_n
        res["cpu_oracle"] = {"value": nb / (t2 - t0) / 1e9, "unit": "GB/s", "cores": 1,
                             "sample": f"first {cpu_n} particles of the frame, compress "
                                       f"{nb / (t1 - t0) / 1e9:.4f} GB/s, decompress "
                                       f"{nb / (t2 - t1) / 1e9:.4f} GB/s"}
    del plan, out, dec
    torch.cuda.empty_cache()
    return res


def bench_batched(args, torch, lcp, datagen, dev):
    """Independent frames of uneven size: one batched lcp_compress / lcp_decompress
    call for all of them against one call per frame (the plain form), same plan
    parameters, same bytes."""
    xs = datagen.batched_frames(args.batched_frames, 14, 22, seed=4)
    sizes = [x.shape[1] for x in xs]
    ntot = int(sum(sizes))
    frames = [torch.from_numpy(x).to(dev) for x in xs]
    del xs
    torch.cuda.synchronize()
    size_d = 12 * ntot
    big = int(np.argmax(sizes))
    bplan = lcp.Plan(args.eb, lcp.EB_REL_GLOBAL, block_log2=-1, sample=frames[big],
                     max_particles=max(sizes), max_batch_particles=ntot,
                     max_batch_frames=len(frames))
    k = bplan.block_log2
    pplan = lcp.Plan(args.eb, lcp.EB_REL_GLOBAL, block_log2=k, max_particles=max(sizes),
                     max_batch_frames=1)
    cap = sum((bplan.bound(n) + 3) & ~3 for n in sizes)
    outb = torch.empty(cap, dtype=torch.uint8, device=dev)
    outp = torch.empty(cap, dtype=torch.uint8, device=dev)
    decb = [torch.empty((3, n), dtype=torch.float32, device=dev) for n in sizes]

    def batched():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, offs, _, _ = bplan.compress(frames, out=outb)
        t1 = time.perf_counter()
        bplan.decompress(outb, offs, outs=decb)
        torch.cuda.synchronize()
        return t1 - t0, time.perf_counter() - t1, offs

    def plain():
        torch.cuda.synchronize()
        offs, lat_c, lat_d = [0], [], []
        for f in frames:
            t = time.perf_counter()
            _, o, _, _ = pplan.compress([f], out=outp[offs[-1]:])
            lat_c.append(time.perf_counter() - t)
            offs.append(offs[-1] + o[1])
        for j in range(len(frames)):
            t = time.perf_counter()
            pplan.decompress(outp, offs[j:j + 2], outs=[decb[j]])
            torch.cuda.synchronize()
            lat_d.append(time.perf_counter() - t)
        return sum(lat_c), sum(lat_d), offs, lat_c, lat_d

    # launch shape: the autotuner's choice for this batch, then the same calls
    # with graphs switched off for comparison
    tuned, tuned_ms, default_ms = bplan.autotune(frames, outb, reps=1)
    log(f"autotune: {tuned}, {tuned_ms:.2f} ms per batch (defaults {default_ms:.2f} ms)")

    def compress_ms(graphs, reps=3):
        bplan.set_tuning(tuned["tile"], tuned["grid"], tuned["slot_grid"], graphs)
        best = 1e30
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t = time.perf_counter()
            bplan.compress(frames, out=outb)
            best = min(best, time.perf_counter() - t)
        return best * 1e3

    ms_nograph = compress_ms(False)
    ms_graph = compress_ms(True)
    bplan.reset()  # frame sequence numbers start again, as the plain plan's do
    for _ in range(args.batched_warmup):
        batched()
        plain()
    bc = bd = pc = pd = 0.0
    lc_all, ld_all, batch_lat = [], [], []
    for _ in range(args.batched_steps):
        c, d, boffs = batched()
        bc += c
        bd += d
        batch_lat.append(c + d)
        c, d, poffs, lc, ld = plain()
        pc += c
        pd += d
        lc_all += lc
        ld_all += ld
    torch.cuda.synchronize()
    same = boffs == poffs and torch.equal(outb[:boffs[-1]], outp[:poffs[-1]])
    assert same, "batched records differ from per-frame records"
    # error bound on a few frames, against the slot permutation
    chk = [0, 1, big, int(np.argmin(sizes))]
    cplan = lcp.Plan(args.eb, lcp.EB_REL_GLOBAL, block_log2=k, max_particles=max(sizes),
                     max_batch_particles=ntot, max_batch_frames=len(chk))
    out2, offs2, _, perms = cplan.compress([frames[j] for j in chk], want_perm=True)
    dec = cplan.decompress(out2, offs2)
    max_ratio_err = 0.0
    for i, j in enumerate(chk):
        f = frames[j]
        eb_abs = args.eb * (float(f.max()) - float(f.min()))
        err = float((dec[i].double() - f[:, perms[i].long()].double()).abs().max())
        assert err <= eb_abs, (j, err, eb_abs)
        max_ratio_err = max(max_ratio_err, err / eb_abs)
    steps = args.batched_steps
    pct = lambda v, q: float(np.percentile(np.asarray(v) * 1e3, q))  # noqa: E731
    return {
        "workload": f"{len(frames)} independent frames, n log-uniform in [2^14, 2^22] "
                    f"(total {ntot}), even uniform / odd clustered in [0,100)^3, float32 xyz, "
                    f"eb={args.eb:g} x each frame's range, LCP-S, block_log2 {k}",
        "frames": len(frames), "particles": ntot,
        "batched_compress_GBps": size_d * steps / bc / 1e9,
        "batched_decompress_GBps": size_d * steps / bd / 1e9,
        "batched_GBps": size_d * steps / (bc + bd) / 1e9,
        "plain_compress_GBps": size_d * steps / pc / 1e9,
        "plain_decompress_GBps": size_d * steps / pd / 1e9,
        "plain_GBps": size_d * steps / (pc + pd) / 1e9,
        "speedup_vs_plain": (pc + pd) / (bc + bd),
        "batch_latency_ms_p50": pct(batch_lat, 50),
        "plain_compress_call_ms_p50": pct(lc_all, 50), "plain_compress_call_ms_p99": pct(lc_all, 99),
        "plain_decompress_call_ms_p50": pct(ld_all, 50),
        "plain_decompress_call_ms_p99": pct(ld_all, 99),
        "ratio": size_d / boffs[-1], "bytes_equal_plain": bool(same),
        "launch_shape": {"autotuned": tuned, "autotune_best_ms": tuned_ms,
                         "defaults_ms": default_ms,
                         "compress_ms_graph": ms_graph, "compress_ms_no_graph": ms_nograph},
        "path_roofline": {"bound": "hbm",
                          "batched_compress": path_frac((size_d + boffs[-1]) * steps, bc),
                          "batched_decompress": path_frac((size_d + boffs[-1]) * steps, bd),
                          "bytes_rule": "S compress 4FN + C, S decompress C + 4FN"},
        "max_err_over_eb": max_ratio_err, "steps": steps,
    }


def served_frames(torch, dev, sizes, n_frames, seed=5):
    """MD-like streams generated on the device: the first n sites of a near-cubic
    lattice (spacing 1), jitter sigma 0.1, then per-step displacement sigma 0.01."""
    from paper_2411_00761_amd import datagen
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    out = []
    for n in sizes:
        nx, ny, nz = datagen.lattice_dims(int(n))
        i = torch.arange(int(n), device=dev, dtype=torch.int64)
        base = torch.stack([(i % nx), (i // nx) % ny, i // (nx * ny)]).to(torch.float32)
        x = base + 0.1 * torch.randn(base.shape, generator=g, device=dev)
        fr = []
        for _ in range(n_frames):
            fr.append(x.clone())
            x = x + 0.01 * torch.randn(base.shape, generator=g, device=dev)
        out.append(fr)
    return out


def bench_served(args, torch, lcp, datagen, dev):
    """Streams served with overlap (lcp_server, several workers) against the plain
    per-call form (one request at a time), on the same Poisson arrival trace."""
    sizes = [int(n) for n in datagen.serve_stream_sizes(args.served_streams, 16, 24, seed=5)]
    T = args.served_frames
    frames = served_frames(torch, dev, sizes, T)
    torch.cuda.synchronize()
    ebs = [1e-3 if j % 2 == 0 else 1e-4 for j in range(len(sizes))]
    caps = [40 * n + 4096 for n in sizes]
    recs = [torch.empty(c, dtype=torch.uint8, device=dev) for c in caps]
    decs = [torch.empty((3, n), dtype=torch.float32, device=dev) for n in sizes]
    # request sequence per stream: C0 D0 C1 D1 ...; streams interleaved at random
    rng = np.random.default_rng(5)
    order = np.concatenate([np.full(2 * T, j) for j in range(len(sizes))])
    rng.shuffle(order)
    nxt = [0] * len(sizes)
    reqs = []
    for j in order:
        t = nxt[j]
        nxt[j] += 1
        reqs.append((int(j), t // 2, "C" if t % 2 == 0 else "D"))
    req_bytes = [12 * sizes[j] for j, _, _ in reqs]

    def plans():
        ps = []
        for j, n in enumerate(sizes):
            ps.append((lcp.Plan(ebs[j], lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=16,
                                block_log2=ks[j], max_particles=n),
                       lcp.Plan(ebs[j], lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=16,
                                block_log2=ks[j], max_particles=n)))
        return ps

    # block size per stream from its first frame
    ks = []
    for j, n in enumerate(sizes):
        p = lcp.Plan(ebs[j], lcp.EB_REL_GLOBAL, multi_frame=True, block_log2=-1, max_particles=n,
                     sample=frames[j][0])
        ks.append(p.block_log2)
        del p

    def run_plain(arrivals):
        ps = plans()
        rec_size = [0] * len(sizes)
        lat, sizes_out = [], []
        t0 = time.monotonic()
        for i, (j, t, kind) in enumerate(reqs):
            a = t0 + (arrivals[i] if arrivals is not None else 0.0)
            while time.monotonic() < a:
                pass
            if kind == "C":
                _, offs, _, _ = ps[j][0].compress([frames[j][t]], out=recs[j])
                rec_size[j] = offs[1]
                sizes_out.append(offs[1])
            else:
                ps[j][1].decompress(recs[j], [0, rec_size[j]], outs=[decs[j]])
                torch.cuda.synchronize()
            lat.append(time.monotonic() - a)
        return time.monotonic() - t0, lat, sizes_out

    batch_particles = min(3 * max(sizes), (1 << 32) - 1)

    def run_served(arrivals, workers, batch_frames=0):
        arena = workers * max(lcp.scratch_bytes(max_particles=n) for n in sizes)
        srv = lcp.Server(arena, workers=workers, batch_frames=batch_frames,
                         batch_particles=batch_particles if batch_frames else 0)
        ids = [srv.open_stream(ebs[j], lcp.EB_REL_GLOBAL, batch_size=16, block_log2=ks[j],
                               max_particles=n) for j, n in enumerate(sizes)]
        torch.cuda.synchronize()
        tickets = []
        if arrivals is None:
            srv.hold(True)  # back to back: the whole queue is there from the start
        t0 = time.monotonic()
        for i, (j, t, kind) in enumerate(reqs):
            a = t0 + (arrivals[i] if arrivals is not None else 0.0)
            while time.monotonic() < a:
                pass
            if kind == "C":
                tickets.append(srv.compress(ids[j], frames[j][t], recs[j]))
            else:
                tickets.append(srv.decompress(ids[j], recs[j], 0, caps[j], decs[j]))
        srv.hold(False)
        res = [srv.wait(tk) for tk in tickets]
        wall = max(r["t_end_ns"] for r in res) / 1e9 - t0
        assert all(r["status"] == 0 for r in res), [r for r in res if r["status"]][:3]
        lat = [(r["t_end_ns"] - r["t_submit_ns"]) / 1e9 for r in res]
        sizes_out = [r["bytes"] for r, (_, _, kind) in zip(res, reqs) if kind == "C"]
        counts = srv.counts()
        srv.close()
        return wall, lat, sizes_out, counts

    W, BF = args.served_workers, args.served_batch
    run_plain(None)  # warm-up
    plain_wall, _, plain_sizes = run_plain(None)
    cap_rps = len(reqs) / plain_wall
    served_wall_b2b, _, served_sizes, _ = run_served(None, W)
    assert served_sizes == plain_sizes, "served records differ from the plain form"
    batched_wall_b2b, _, batched_sizes, b2b_counts = run_served(None, W, BF)
    assert batched_sizes == plain_sizes, "batched served records differ from the plain form"
    tot = float(sum(req_bytes))
    pct = lambda v, q: float(np.percentile(np.asarray(v) * 1e3, q))  # noqa: E731
    sweep = []
    for load in args.served_loads:
        rate = load * cap_rps
        arrivals = np.cumsum(np.random.default_rng(11).exponential(1.0 / rate, size=len(reqs)))
        p_wall, p_lat, _ = run_plain(arrivals)
        s_wall, s_lat, _, _ = run_served(arrivals, W)
        b_wall, b_lat, _, b_counts = run_served(arrivals, W, BF)
        sweep.append({"load": load, "arrival_rate_req_per_s": rate,
                      "plain_p50_ms": pct(p_lat, 50), "plain_p99_ms": pct(p_lat, 99),
                      "served_p50_ms": pct(s_lat, 50), "served_p99_ms": pct(s_lat, 99),
                      "batched_p50_ms": pct(b_lat, 50), "batched_p99_ms": pct(b_lat, 99),
                      "plain_GBps": tot / p_wall / 1e9, "served_GBps": tot / s_wall / 1e9,
                      "batched_GBps": tot / b_wall / 1e9, "batched_counts": b_counts})
        log(f"served load {load:g}: p99 plain {sweep[-1]['plain_p99_ms']:.2f} ms, served "
            f"{sweep[-1]['served_p99_ms']:.2f} ms, batched {sweep[-1]['batched_p99_ms']:.2f} ms")
    return {
        "workload": f"{len(sizes)} MD-like streams, n log-uniform in [2^16, 2^24] (total "
                    f"{sum(sizes)}), {T} frames each, eb 1e-3 / 1e-4 x range alternating, "
                    f"requests C,D per frame in random stream order, Poisson arrivals at "
                    f"the listed fractions of the plain form's capacity",
        "requests": len(reqs), "workers": W, "batch_frames": BF,
        "batch_particles": batch_particles,
        "plain_capacity_req_per_s": cap_rps,
        "plain_back_to_back_GBps": tot / plain_wall / 1e9,
        "served_back_to_back_GBps": tot / served_wall_b2b / 1e9,
        "batched_back_to_back_GBps": tot / batched_wall_b2b / 1e9,
        "batched_back_to_back_counts": b2b_counts,
        "sweep": sweep,
        "record_sizes_equal_plain": True,
    }


def bench_next_rows(args, torch, lcp, frames, k, steps=2, n_random=16):
    """The next rows built beyond the hot path, on the trajectory's resident frames:
    int32 fields (the frames as fixed point, 1e-3 lattice units), data of two
    spatial dimensions (x and y), and the random-access container (Sec. 7.3) of the
    float stream's records.  Each leg checks its output before reporting."""
    res = {}
    n, nf = frames[0].shape[1], len(frames)
    dev = frames[0].device
    kw = dict(multi_frame=True, batch_size=args.batch, block_log2=k, max_particles=n)

    def timed(plan, dplan, xs, outbuf, decs, timer=None):
        """One untimed pass, then `steps` timed ones (the kernel timer, if named, over those)."""
        tc = td = 0.0
        for rep in range(steps + 1):
            if rep == 1 and timer:
                plan.timer_set(timer)
            plan.reset()
            dplan.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out, offs, used, _ = plan.compress(xs, out=outbuf)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            dplan.decompress(out, offs, outs=decs)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if rep:
                tc += t1 - t0
                td += t2 - t1
        return tc / steps, td / steps, out, offs, used

    # int32 fields: the trajectory in fixed point (rounded to nearest), relative bound as the
    # float leg's; the run kernel's integer instance timed
    ints = [(f.double() * 1000.0).round().to(torch.int32) for f in frames]
    plan = lcp.Plan(args.eb, lcp.EB_REL_GLOBAL, dtype=lcp.DTYPE_I32, **kw)
    dplan = lcp.Plan(args.eb, lcp.EB_REL_GLOBAL, dtype=lcp.DTYPE_I32, **kw)
    cap = sum((plan.bound(n) + 3) & ~3 for _ in ints)
    outbuf = torch.empty(cap, dtype=torch.uint8, device=dev)
    decs = [torch.empty((3, n), dtype=torch.int32, device=dev) for _ in ints]
    tc, td, out, offs, used = timed(plan, dplan, ints, outbuf, decs, "t_resid_run/1")
    kms, kl, kb = plan.timer_read()
    eb_i = args.eb * float(int(ints[0].max()) - int(ints[0].min()))
    chk = lcp.Plan(args.eb, lcp.EB_REL_GLOBAL, dtype=lcp.DTYPE_I32, **kw)
    o2, of2, _, perms = chk.compress(ints[:3], want_perm=True)
    dchk = lcp.Plan(args.eb, lcp.EB_REL_GLOBAL, dtype=lcp.DTYPE_I32, **kw)
    d2 = dchk.decompress(o2, of2)
    err = max(int((d2[j].long() - ints[j][:, perms[j].long()].long()).abs().max()) for j in range(3))
    assert err <= eb_i, (err, eb_i)
    size_i = sum(x.numel() * 4 for x in ints)
    achieved = kb / (kms * 1e-3) / 1e9 if kl else None
    res["int32"] = {
        "workload": f"the trajectory's {nf} frames as int32 fixed point (1e-3 lattice units), "
                    f"eb={args.eb:g} x range, batch {args.batch}, LCP-FSM S/T",
        "compress_GBps": size_i / tc / 1e9, "decompress_GBps": size_i / td / 1e9,
        "GBps": size_i / (tc + td) / 1e9, "ratio": size_i / offs[-1],
        "temporal_frames": sum(1 for u in used if u == lcp.METHOD_T),
        "max_abs_err": err, "eb_abs": eb_i,
        "run_kernel": {"launches": kl, "avg_launch_us": kms / kl * 1e3 if kl else None,
                       "achieved_GBps": achieved,
                       "frac": achieved / HBM_PEAK_GBPS if achieved else None}}
    del ints, plan, dplan, chk, dchk, outbuf, decs, o2, d2
    torch.cuda.empty_cache()

    # two spatial dimensions: x and y of every frame
    xy = [f[:2] for f in frames]
    plan = lcp.Plan(args.eb, lcp.EB_REL_GLOBAL, n_fields=2, n_dims=2, **kw)
    dplan = lcp.Plan(args.eb, lcp.EB_REL_GLOBAL, n_fields=2, n_dims=2, **kw)
    cap = sum((plan.bound(n) + 3) & ~3 for _ in xy)
    outbuf = torch.empty(cap, dtype=torch.uint8, device=dev)
    decs = [torch.empty((2, n), dtype=torch.float32, device=dev) for _ in xy]
    tc, td, out, offs, used = timed(plan, dplan, xy, outbuf, decs)
    size_2 = sum(x.numel() * 4 for x in xy)
    res["two_dims"] = {
        "workload": f"x and y of the trajectory's {nf} frames (n_dims = 2), eb={args.eb:g} x range",
        "compress_GBps": size_2 / tc / 1e9, "decompress_GBps": size_2 / td / 1e9,
        "GBps": size_2 / (tc + td) / 1e9, "ratio": size_2 / offs[-1],
        "temporal_frames": sum(1 for u in used if u == lcp.METHOD_T)}
    del plan, dplan, outbuf, decs
    torch.cuda.empty_cache()

    # the container: the float stream's records packed; one sequential retrieval of every
    # frame, then single-frame requests in random order, each checked against the
    # sequential decode
    plan = lcp.Plan(args.eb, lcp.EB_REL_GLOBAL, **kw)
    dplan = lcp.Plan(args.eb, lcp.EB_REL_GLOBAL, **kw)
    out, offs, _, _ = plan.compress(frames)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cbuf = lcp.Container.pack(out, offs, args.batch)
    torch.cuda.synchronize()
    t_pack = time.perf_counter() - t0
    cont = lcp.Container(cbuf)
    seq = [torch.empty((3, n), dtype=torch.float32, device=dev) for _ in range(nf)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dec_all = cont.retrieve(dplan, list(range(nf)), seq)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    rng = np.random.default_rng(7)
    picks = [int(v) for v in rng.integers(0, nf, size=n_random)]
    one = torch.empty((3, n), dtype=torch.float32, device=dev)
    lat, decoded = [], []
    for fidx in picks:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        decoded.append(cont.retrieve(dplan, [fidx], [one]))
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        assert torch.equal(one.view(torch.int32), seq[fidx].view(torch.int32)), fidx
    size_d = sum(f.numel() * 4 for f in frames)
    res["container"] = {
        "workload": f"the float trajectory's {nf} records (batch {args.batch}) packed for "
                    f"random access",
        "frames": nf, "anchors": cont.anchors, "container_bytes": cbuf.numel(),
        "pack_ms": t_pack * 1e3,
        "retrieve_all_GBps": size_d / t_all / 1e9, "retrieve_all_records_decoded": dec_all,
        "single_frame_requests": n_random,
        "single_frame_ms_p50": float(np.percentile(np.array(lat) * 1e3, 50)),
        "single_frame_ms_max": float(np.max(lat) * 1e3),
        "records_decoded_per_request_mean": float(np.mean(decoded)),
        "records_decoded_per_request_max": int(np.max(decoded)),
        "checked": "every single-frame request equals the sequential retrieval bit for bit"}
    cont.close()
    del cbuf, seq, one

    # the dictionary stage (lcp_dict_*) over the float stream's records, then over
    # the records of frames that do not move (frame 0 eight times: every temporal
    # residual is zero, one Huffman bit per value); each stream decoded and checked
    def dict_leg(recs, what, reps=3, bl=16):
        nbytes = recs.numel()
        scr_e = torch.empty(lcp.dict_scratch_bytes(nbytes, bl, True), dtype=torch.uint8, device=dev)
        scr_d = torch.empty(lcp.dict_scratch_bytes(nbytes, bl, False), dtype=torch.uint8, device=dev)
        sout = torch.empty(lcp.dict_bound(nbytes, bl), dtype=torch.uint8, device=dev)
        back = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        te, td = [], []
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, ssize = lcp.dict_encode(recs, block_log2=bl, out=sout, scratch=scr_e)
            t1 = time.perf_counter()
            lcp.dict_decode(sout, ssize, nbytes, block_log2=bl, out=back, scratch=scr_d)
            torch.cuda.synchronize()
            te.append(t1 - t0)
            td.append(time.perf_counter() - t1)
        assert torch.equal(back, recs), what
        te, td = sorted(te[1:])[reps // 2], sorted(td[1:])[reps // 2]
        return {"workload": what, "block_log2": bl, "input_bytes": nbytes, "stream_bytes": ssize,
                "size_ratio": ssize / nbytes, "encode_GBps": nbytes / te / 1e9,
                "decode_GBps": nbytes / td / 1e9, "checked": "decoded stream equals the records"}

    recs = out[:offs[-1]]
    res["dictionary"] = dict_leg(recs, f"the float trajectory's {nf} records "
                                       f"({offs[-1]} bytes, CR {size_d / offs[-1]:.2f})")
    res["dictionary"]["ratio_with_stage"] = size_d / res["dictionary"]["stream_bytes"]
    still = [frames[0]] * 8
    plan.reset()
    out8, offs8, used8, _ = plan.compress(still)
    size_8 = sum(f.numel() * 4 for f in still)
    res["dictionary_static"] = dict_leg(out8[:offs8[-1]], "frame 0 eight times (particles that "
                                        f"do not move; CR {size_8 / offs8[-1]:.2f} before the stage: "
                                        "the temporal records are a few bytes each, the spatial "
                                        "record is the rest)")
    res["dictionary_static"]["ratio_with_stage"] = size_8 / res["dictionary_static"]["stream_bytes"]
    del plan, dplan, out, out8
    torch.cuda.empty_cache()
    return res


def measured_traffic(kernel):
    """HBM bytes per launch from the committed counter summary, if it was taken on
    the current kernel sources (else None)."""
    from paper_2411_00761_amd import profiling
    path = os.path.join(ROOT, "profiles", f"{kernel}_traffic.json")
    try:
        t = json.load(open(path))
    except (OSError, ValueError):
        return None
    if t.get("kernel") != kernel or t.get("source_sha256") != profiling.source_hash():
        return None
    return t["traffic_bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--frames", type=int, default=64)
    ap.add_argument("--n", type=int, default=1 << 22)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--eb", type=float, default=1e-4)
    ap.add_argument("--cpu-frames", type=int, default=6,
                    help="frames of the trajectory the oracle codes for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--roofline-kernel", default=ROOFLINE_KERNEL)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run three 256 MiB device copies (counter calibration)")
    ap.add_argument("--workloads", default="md,next,c1,c3,batched,served",
                    help="comma list: md (the trajectory, the headline value), next (int32 "
                         "fields, two dimensions and the container on the trajectory's frames; "
                         "needs md), c1 (uniform frame), c3 (cosmology snapshot), batched, served")
    ap.add_argument("--c3-n", type=int, default=1 << 27)
    ap.add_argument("--c3-steps", type=int, default=3)
    ap.add_argument("--c3-timer", default="radix_scatter")
    ap.add_argument("--c1-steps", type=int, default=20)
    ap.add_argument("--batched-frames", type=int, default=256)
    ap.add_argument("--batched-steps", type=int, default=3)
    ap.add_argument("--batched-warmup", type=int, default=1)
    ap.add_argument("--served-streams", type=int, default=32)
    ap.add_argument("--served-frames", type=int, default=6)
    ap.add_argument("--served-workers", type=int, default=4)
    ap.add_argument("--served-loads", type=lambda v: [float(x) for x in v.split(",")],
                    default=[0.3, 0.6, 0.9, 1.5], help="arrival rates as fractions of plain capacity")
    ap.add_argument("--served-batch", type=int, default=16,
                    help="requests one merged launch set takes in the batched served leg")
    args = ap.parse_args()
    work = args.workloads.split(",")

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "bench.py measures one GPU: run with --gpus 1 (whole "
                                   "batches of frames would shard across GPUs; that path is "
                                   "not implemented)"}))
        sys.exit(2)

    import torch

    from paper_2411_00761_amd import datagen, lcp

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    result = {"metric": METRIC, "value": None, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True,
              "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic"}
    ceiling = copy_ceiling(torch, dev)
    log(f"copy ceiling {ceiling['copy_GBps']:.0f} GB/s, read {ceiling['read_GBps']:.0f} GB/s")

    if "md" in work:
        nx, ny, nz = (256, 128, 128) if args.n == 1 << 22 else datagen.lattice_dims(args.n)
        log(f"generating {args.frames} frames of {args.n} particles")
        traj = datagen.MDTrajectory(args.n, dims=(nx, ny, nz), seed=2)
        frames_np, frames = [], []
        for j in range(args.frames):
            f = traj.next_frame()
            if j < args.cpu_frames:
                frames_np.append(f)
            frames.append(torch.from_numpy(f).to(dev))
        torch.cuda.synchronize()
        size_d = sum(f.numel() * 4 for f in frames)

        plan = lcp.Plan(args.eb, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=args.batch,
                        block_log2=-1, max_particles=args.n, sample=frames[0])
        k = plan.block_log2
        dplan = lcp.Plan(args.eb, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=args.batch,
                         block_log2=k, max_particles=args.n)
        log(f"block_log2 k={k}")
        cap = sum((plan.bound(args.n) + 3) & ~3 for _ in frames)
        outbuf = torch.empty(cap, dtype=torch.uint8, device=dev)
        decbufs = [torch.empty((3, args.n), dtype=torch.float32, device=dev) for _ in range(args.frames)]

        def step():
            plan.reset()
            dplan.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out, offs, used, _ = plan.compress(frames, out=outbuf)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            dplan.decompress(out, offs, outs=decbufs)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            return t1 - t0, t2 - t1, offs, used

        for w in range(args.warmup):
            step()
            log(f"warmup {w} done")
        # every launch of the run kernel is timed (a few per step)
        plan.timer_set(f"{args.roofline_kernel}/1")
        dplan.timer_set(f"{args.roofline_kernel}/1")
        tc = td = 0.0
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for s_ in range(args.steps):
            c, d, offs, used = step()
            tc += c
            td += d
            log(f"step {s_}: compress {c * 1e3:.1f} ms, decompress {d * 1e3:.1f} ms")
        torch.cuda.synchronize()
        t_total = time.perf_counter() - t_start
        kms, klaunch, kbytes = plan.timer_read()
        dkms, dklaunch, dkbytes = dplan.timer_read()
        kms, klaunch, kbytes = kms + dkms, klaunch + dklaunch, kbytes + dkbytes

        comp_bytes = offs[-1]
        ratio = size_d / comp_bytes
        n_t = sum(1 for u in used if u == lcp.METHOD_T)
        # algorithmic bytes of one step, per frame by its method: spatial 4FN + C both ways,
        # temporal 12FN + 4N + C to compress and 12FN + C to decompress
        bc = bd = 0
        for j, u in enumerate(used):
            c = offs[j + 1] - offs[j]
            if u == lcp.METHOD_T:
                bc += t_bytes_c(3, args.n, c)
                bd += t_bytes_d(3, args.n, c)
            else:
                bc += s_bytes(3, args.n, c)
                bd += s_bytes(3, args.n, c)
        # error bound check on a few frames against the slot permutation
        eb_abs = args.eb * (float(frames[0].max()) - float(frames[0].min()))
        chk = lcp.Plan(args.eb, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=args.batch,
                       block_log2=k, max_particles=args.n)
        nchk = min(3, len(frames))
        out2, offs2, _, perms = chk.compress(frames[:nchk], want_perm=True)
        dchk = lcp.Plan(args.eb, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=args.batch,
                        block_log2=k, max_particles=args.n)
        dec = dchk.decompress(out2, offs2)
        max_err = max(float((dec[j].double() - frames[j][:, perms[j].long()].double()).abs().max())
                      for j in range(nchk))
        assert max_err <= eb_abs, (max_err, eb_abs)
        del chk, dchk, dec, out2

        if args.copy_probe:
            src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            del src, dst

        achieved = (kbytes / klaunch) / (kms / klaunch * 1e-3) / 1e9 if klaunch else None
        # what the run kernel itself reads and writes per launch: J (4F + F) + 4 + 8F bytes
        # per particle (J frames read and their residual bytes written; the permutation and
        # the first reference codes read and the last codes written once), F = 3
        own = ((kbytes / klaunch) / (4 + 12 * 3) * (5 * 3) + args.n * (4 + 8 * 3)) if klaunch \
            else None
        own_gbps = own / (kms / klaunch * 1e-3) / 1e9 if klaunch else None
        result.update({
            "value": size_d * args.steps / (tc + td) / 1e9,
            "ms_per_step": t_total / args.steps * 1e3,
            "config": {"workload": f"MD-like trajectory, {args.frames} frames x {args.n} particles "
                                   f"({nx}x{ny}x{nz} lattice, jitter 0.1, step 0.01), float32 xyz, "
                                   f"eb={args.eb:g} x range, batch {args.batch}, LCP-FSM S/T",
                       "frames": args.frames, "particles_per_frame": args.n, "block_log2": k,
                       "chunk_log2": 10},
            "compress_GBps": size_d * args.steps / tc / 1e9,
            "decompress_GBps": size_d * args.steps / td / 1e9,
            "ratio": ratio,
            "bits_per_value": 32.0 / ratio,
            "temporal_frames": n_t,
            "max_abs_err": max_err,
            "eb_abs": eb_abs,
            "roofline": {"bound": "hbm", "kernel": args.roofline_kernel,
                         "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": (achieved / HBM_PEAK_GBPS) if achieved else None,
                         "traffic": measured_traffic(args.roofline_kernel),
                         "timed_launches": klaunch, "timed_every": 1,
                         "avg_launch_us": (kms / klaunch * 1e3) if klaunch else None,
                         "own_bytes_per_launch": own, "own_GBps": own_gbps,
                         "own_frac": (own_gbps / HBM_PEAK_GBPS) if own_gbps else None,
                         "own_vs_copy_ceiling": (own_gbps / ceiling["copy_GBps"])
                         if own_gbps else None,
                         "bytes_per_launch": (kbytes / klaunch) if klaunch else None,
                         "bytes_rule": "4 + 12F per particle and frame (a frame, its reference "
                                       "codes and the slot permutation read, its codes written) "
                                       "times the J frames of the launch; the run kernel keeps "
                                       "the codes in registers and itself moves J(4F + F) + 4 + "
                                       "8F bytes per particle (own_bytes_per_launch), so frac, "
                                       "on the per-frame figure, can pass 1 where own_frac "
                                       "cannot",
                         "copy_ceiling": ceiling, "mall_note": MALL_NOTE},
            "path_roofline": {"bound": "hbm",
                              "compress": path_frac(bc * args.steps, tc),
                              "decompress": path_frac(bd * args.steps, td),
                              "bytes_rule": "per frame: S 4FN + C both ways; T compress "
                                            "12FN + 4N + C, T decompress 12FN + C",
                              "mall_note": MALL_NOTE},
        })
        # Sec. 7.4.2: the same frames with anchors at eb / 5 while correlated
        splan = lcp.Plan(args.eb, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=args.batch,
                         block_log2=k, max_particles=args.n, anchor_scale=5)
        sdplan = lcp.Plan(args.eb, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=args.batch,
                          block_log2=k, max_particles=args.n, anchor_scale=5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out5, offs5, used5, perms5 = splan.compress(frames, out=outbuf, want_perm=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dec5 = sdplan.decompress(out5, offs5, outs=decbufs)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        err5 = max(float((dec5[j].double() - frames[j][:, perms5[j].long()].double()).abs().max())
                   for j in range(0, len(frames), 7))
        assert err5 <= eb_abs, (err5, eb_abs)
        result["anchor_scale"] = {
            "scale": 5, "ratio": size_d / offs5[-1], "ratio_without": ratio,
            "temporal_frames": sum(1 for u in used5 if u == lcp.METHOD_T),
            "compress_GBps": size_d / (t1 - t0) / 1e9, "decompress_GBps": size_d / (t2 - t1) / 1e9,
            "max_abs_err": err5, "note": "one untimed-warmup-free pass; every 7th frame checked"}
        log(f"anchor scale 5: ratio {size_d / offs5[-1]:.3f} (without {ratio:.3f})")
        del splan, sdplan, dec5, out5, perms5
        if "next" in work:
            log("int32 fields, two dimensions, container")
            result["next_rows"] = bench_next_rows(args, torch, lcp, frames, k)
            log(json.dumps(result["next_rows"]))
        if not args.no_cpu_baseline:
            log(f"cpu baseline: oracle on {len(frames_np)} frames")
            cb = cpu_baseline(frames_np, args.eb, args.batch, k, list(used), 12 * args.n)
            result["cpu_baseline"] = cb
        del frames, decbufs, outbuf, plan, dplan
        torch.cuda.empty_cache()
    if "c1" in work:
        log("uniform frame (2^18 particles)")
        x = torch.from_numpy(datagen.uniform_frame(1 << 18, seed=1)).to(dev)
        result["c1"] = bench_single_s(args, torch, lcp, "uniform frame, 262144 particles in "
                                      "[0,100)^3, float32 xyz, eb=1e-3 absolute, LCP-S",
                                      x, lcp.EB_ABS, 1e-3, args.c1_steps, 3, "decode_huff", 0)
        log(json.dumps(result["c1"]))
        del x
    if "c3" in work:
        log(f"cosmology snapshot ({args.c3_n} particles x 6 fields)")
        x = datagen.cosmology_snapshot_device(torch, args.c3_n, dev)
        torch.cuda.synchronize()
        result["c3"] = bench_single_s(
            args, torch, lcp, f"cosmology-like snapshot, {args.c3_n} particles: 2000 Gaussian "
            f"halos (sigma log-uniform 0.1-2.0) + 30% uniform in [0,256)^3, shuffled, velocities "
            f"N(0, 300^2), float32 x 6 fields, eb=1e-4 x range per field, LCP-S",
            x, lcp.EB_REL_PER_FIELD, 1e-4, args.c3_steps, 1, args.c3_timer,
            0 if args.no_cpu_baseline else 1 << 22)
        log(json.dumps(result["c3"]))
        del x
        torch.cuda.empty_cache()
    if "batched" in work:
        torch.cuda.empty_cache()
        log("batched workload")
        result["batched"] = bench_batched(args, torch, lcp, datagen, dev)
        log(json.dumps(result["batched"]))
    if "served" in work:
        torch.cuda.empty_cache()
        log("served workload")
        result["served"] = bench_served(args, torch, lcp, datagen, dev)
        log(json.dumps(result["served"]))
    print(json.dumps(result))


if __name__ == "__main__":
    main()
