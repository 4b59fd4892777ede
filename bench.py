#!/usr/bin/env python3
"""Benchmark of the clip-alignment hot path on one MI355X.

Workload: 50,000 clips of 128 x 128 from 1,000 templates of 6-24 rectangles,
edge jitter +-4 px, pattern offsets +-16 px, marker half-window 16 (33 x 33
shifts); cosine threshold 19/20 and edge tolerance 3 px.  Inputs are seeded
and synthetic; the rectangle lists are resident in HBM before timing starts.

One step is one pass of the hot path over the clip set:
  rasterise + pack + FP64 spectra (ca_clips_create), cosine candidate
  generation (ca_prune), mixed-precision alignment with FP64 re-decision of
  near ties (ca_align_pairs), edge candidate generation and edge-track
  alignment.
`value` counts the unordered cosine pairs carried through alignment per second
of the whole step.  Beside it the JSON line carries the roofline of the
dominant kernel, the plain FP32 per-pair kernel on the same pair list, the
edge track's rate, the run-time FP64 check of decided pairs, the mixed-size
workload (200,000 clips of 64/128/256, windows 4..32, 41.3M pairs) in one
autotuned call, serving, and the FP64 oracle timed on this host's cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# 32-bit integer vector operations: 256 CUs x 4 SIMDs x 16 lanes a clock at 2.4 GHz
INT_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
PROFILE = os.path.join(ROOT, "profiles", "c128_bench_hbm_counters.md")
KERNEL_SOURCES = ["paper_2512_13133_amd/csrc/pcm_mfma.hip", "paper_2512_13133_amd/csrc/mfma_common.h",
                  "paper_2512_13133_amd/csrc/pair_common.h", "paper_2512_13133_amd/csrc/internal.h"]


def profiled_traffic(kernel):
    """Scaled HBM bytes per launch of `kernel` from the committed counter summary,
    or None when the summary is missing or the kernel's sources changed since."""
    import hashlib
    import re
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for src in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    m = re.search(r"sha256 of [^:]*: ([0-9a-f]{64})", text)
    if not m or m.group(1) != h.hexdigest():
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip("|").split("|")]
        if len(cells) == 5 and cells[0] == "ca::" + kernel:
            return float(cells[4]) * 1e9
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--path", default="mixed", choices=["mixed", "fp32", "fp64"])
    ap.add_argument("--clips", type=int, default=50_000)
    ap.add_argument("--templates", type=int, default=1_000)
    ap.add_argument("--no-edge", action="store_true", help="skip the edge track (diagnostics only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-comparator", action="store_true", help="skip the plain FP32 comparator")
    ap.add_argument("--no-xcorr", action="store_true", help="skip the exact-objective alignment")
    ap.add_argument("--no-xysep", action="store_true", help="skip the XY-separation alignment")
    ap.add_argument("--no-mixed-sizes", action="store_true", help="skip the mixed-size workload")
    ap.add_argument("--no-schedule-study", action="store_true", help="skip the relaxation-schedule study")
    ap.add_argument("--no-contour", action="store_true", help="skip the edge track over full boundary edges")
    ap.add_argument("--scale-clusters", action="store_true",
                    help="only run the method end to end on the 2M-clip workload (cosine 19/20 and the edge track "
                         "over full boundary edges at 2 px, K = 3; box edges at 2 px, K = 1) and print its object "
                         "(several minutes)")
    ap.add_argument("--scale-tracks", default="cosine,contour,edge",
                    help="tracks of --scale-clusters, comma-separated (cosine, contour, edge)")
    ap.add_argument("--mixed-sizes-only", action="store_true",
                    help="only run the mixed-size workload (profiling) and print its object")
    ap.add_argument("--serve-library", type=int, default=100_000)
    ap.add_argument("--serve-seconds", type=float, default=8.0)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.scale_clusters:
        print(json.dumps({"scale_clusters": scale_clusters(tuple(args.scale_tracks.split(",")))}))
        return
    if args.mixed_sizes_only:
        import paper_2512_13133_amd as ca
        print(json.dumps({"mixed_sizes": mixed_sizes_bench(ca.Context(0))}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; sharding across GPUs is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import clipgen
    import paper_2512_13133_amd as ca

    dev = torch.device("cuda", 0)
    t0 = time.time()
    cs = clipgen.c128(n_clips=args.clips, n_templates=args.templates)
    log(f"[bench] generated {cs.n} clips in {time.time() - t0:.1f}s")
    d_ptr = torch.from_numpy(cs.rect_ptr).to(dev)
    d_rects = torch.from_numpy(cs.rects.reshape(-1).copy()).to(dev)
    d_n = torch.from_numpy(cs.raster_n).to(dev)
    d_w = torch.from_numpy(cs.marker_w).to(dev)
    ctx = ca.Context(0)
    lib = ctx.lib
    P = ca.P
    import ctypes as C

    # the read bandwidth a plain streaming kernel reaches on this device (best
    # of three rounds of ten reads of a 4 GiB buffer, before the workload's
    # allocations), beside which the main kernel's read rate is set
    probe_buf = torch.empty(1 << 30, dtype=torch.float32, device=dev)
    probe_ms = min(ca.probe_read_bandwidth(probe_buf, reps=10) for _ in range(3))
    read_probe = {"bytes": probe_buf.numel() * 4, "GBps": round(probe_buf.numel() * 4 / (probe_ms * 1e-3) / 1e9, 1),
                  "kernel": "ca_probe_read_bandwidth: sixteen 16-byte loads in flight per thread"}
    del probe_buf
    torch.cuda.empty_cache()

    def make_clips(fp32=False, contours=False):
        h = P()
        flags = ca.CA_CLIPS_DEVICE_PTRS | (ca.CA_CLIPS_FP32 if fp32 else 0) | (ca.CA_CLIPS_CONTOURS if contours else 0)
        ctx._check(lib.ca_clips_create(ctx.h, ctx._stream(), cs.n, d_ptr.data_ptr(), d_rects.data_ptr(),
                                       d_n.data_ptr(), d_w.data_ptr(), flags, C.byref(h)))
        return ca.ClipSet(ctx, h, cs.n)

    stage_t = {}

    def timed(name, fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        stage_t[name] = stage_t.get(name, 0.0) + time.perf_counter() - t
        return r

    def step(keep=False):
        # FP32 spectra serve the FP32 path and the FP32 screen of the mixed path's re-decision
        h = timed("clips", lambda: make_clips(args.path != "fp64"))
        rep, mem = timed("prune_cosine", lambda: ctx.prune(h, "cosine", (19, 20)))
        out = timed("align_cosine", lambda: ctx.align_pairs(h, rep, mem, "cosine", (19, 20), args.path))
        n_e = 0
        if not args.no_edge:
            rep_e, mem_e = timed("prune_edge", lambda: ctx.prune(h, "edge", 3))
            timed("align_edge", lambda: ctx.align_pairs(h, rep_e, mem_e, "edge", 3))
            n_e = rep_e.numel()
            del rep_e, mem_e
        res = (h, rep, mem, out) if keep else None
        if not keep:
            h.close()
        return rep.numel(), n_e, res

    for w in range(args.warmup):
        n_c, n_e, _ = step()
        log(f"[bench] warmup {w}: cosine pairs {n_c}, edge pairs {n_e}")
    stage_t.clear()
    ctx.reset_stats()
    torch.cuda.synchronize()
    t = time.perf_counter()
    tot_c = tot_e = 0
    last = None
    for s in range(args.steps):
        n_c, n_e, last = step(keep=(s == args.steps - 1))
        tot_c += n_c
        tot_e += n_e
        log(f"[bench] step {s}: cosine pairs {n_c}, edge pairs {n_e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    st = ctx.stats()
    ms_per_step = elapsed * 1000.0 / args.steps
    value = tot_c / elapsed

    # dominant kernel of the cosine path: HIP events recorded by the library on
    # the launch stream around each launch of the main alignment kernel
    main_ms = st["t_main_ms"] / max(st["n_main_launch"], 1)
    main_bytes = st["main_alg_bytes"] / max(st["n_main_launch"], 1)
    achieved = main_bytes / (main_ms * 1e-3) / 1e9
    roofline = {"kernel": "pcm_mfma128_kernel" if args.path == "mixed" else "pcm_fft_kernel",
                "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": profiled_traffic("pcm_mfma128_kernel") if args.path == "mixed" else None,
                "avg_launch_ms": round(main_ms, 3), "alg_bytes_per_launch": main_bytes}
    read_probe["main_kernel_frac"] = round(achieved / read_probe["GBps"], 4)

    h, rep, mem, out = last
    n_pairs = rep.numel()
    kernel_rate = n_pairs / (main_ms * 1e-3) if main_ms > 0 else None
    # plain FP32 per-pair comparator on the identical pair list
    comparator = None
    if args.path == "mixed" and not args.no_comparator:
        h32 = h  # the step's clip set holds FP32 spectra
        ctx.align_pairs(h32, rep, mem, "cosine", (19, 20), "fp32")  # warm
        ctx.reset_stats()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        out32 = ctx.align_pairs(h32, rep, mem, "cosine", (19, 20), "fp32")
        torch.cuda.synchronize()
        call_s = time.perf_counter() - t1
        st32 = ctx.stats()
        same = all(bool(torch.equal(out[k], out32[k])) for k in ("bits", "shift", "count", "score"))
        # the per-pair FFT reads both clips' FP32 spectra and bits; a batched
        # FP32 design would read only the member's (the representative staged
        # once per run), so its HBM floor is the fair bound to compare against
        b32 = 2 * 128 * 65 * 8 + 2 * 2048
        b32_batched = 128 * 65 * 8 + 2048
        floor_ms = n_pairs * b32_batched / (HBM_PEAK_GBS * 1e9) * 1e3
        comparator = {"path": "fp32 per-pair FFT", "kernel_pairs_per_s": n_pairs / (st32["t_main_ms"] * 1e-3),
                      "call_pairs_per_s": n_pairs / call_s, "identical_results": same,
                      "kernel_ms": st32["t_main_ms"], "rescored": st32["pairs_rescored"],
                      "own_hbm_frac": round(n_pairs * b32 / (st32["t_main_ms"] * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
                      "batched_fp32_hbm_floor_ms": round(floor_ms, 1),
                      "main_kernel_vs_batched_fp32_floor": round(floor_ms / main_ms, 2)}
    # exact-objective alignment (largest overlap count over the window) on the
    # same pair list: integer AND / bit-count work on the vector ALUs
    xcorr = None
    if args.path == "mixed" and not args.no_xcorr:
        ox = ctx.align_pairs(h, rep, mem, "cosine", (19, 20), "xcorr")  # warm
        ctx.reset_stats()
        ox = ctx.align_pairs(h, rep, mem, "cosine", (19, 20), "xcorr")
        torch.cuda.synchronize()
        stx = ctx.stats()
        xms = stx["t_main_ms"]
        # algorithmic work: AND + bit count per 32-bit word of every row at every
        # window shift (33 x 33 at half-window 16), one surface for both directions
        ops = float(n_pairs) * 33 * 33 * 128 * 4 * 2
        xcorr = {"path": "exact objective (largest overlap count)", "kernel_ms": round(xms, 3),
                 "pairs_per_s": n_pairs / (xms * 1e-3),
                 "count_never_below_phase_correlation": bool((ox["count"] >= out["count"]).all()),
                 "shift_differs_from_phase_correlation": int((ox["shift"] != out["shift"]).any(dim=2).any(dim=1).sum()),
                 "roofline": {"kernel": "xcorr_kernel", "bound": "alu", "achieved": round(ops / (xms * 1e-3) / 1e12, 2),
                              "peak": INT_PEAK_TOPS, "unit": "Tops/s",
                              "frac": round(ops / (xms * 1e-3) / 1e12 / INT_PEAK_TOPS, 4),
                              "ops_per_pair": 33 * 33 * 128 * 4 * 2}}
        del ox
    # XY-separation alignment (interval competition, Sec. 3.2.1(2)) on the same
    # pair list: integer geometry and one overlap count per direction, set
    # against the phase-correlation cover of the step
    xysep = None
    if args.path == "mixed" and not args.no_xysep:
        oy = ctx.align_pairs(h, rep, mem, "cosine", (19, 20), "xysep")  # warm
        ctx.reset_stats()
        oy = ctx.align_pairs(h, rep, mem, "cosine", (19, 20), "xysep")
        torch.cuda.synchronize()
        yms = ctx.stats()["t_main_ms"]

        def n_dirs(b):
            return int((b & 1).sum().item() + ((b >> 1) & 1).sum().item())

        # algorithmic bytes: both clips' bit rasters (2,048 B each) and polygon
        # box tables (512 B each)
        yb = 2 * 2048 + 2 * 512
        xysep = {"path": "XY-separation interval competition", "kernel_ms": round(yms, 3),
                 "pairs_per_s": n_pairs / (yms * 1e-3),
                 "speedup_vs_phase_correlation_kernel": round(main_ms / yms, 2),
                 "covering_directions": n_dirs(oy["bits"]),
                 "covering_directions_phase_correlation": n_dirs(out["bits"]),
                 "covering_both": n_dirs(oy["bits"] & out["bits"]),
                 "directions_same_shift": int((oy["shift"] == out["shift"]).all(dim=2).sum().item()),
                 "alg_bytes_per_pair": yb, "achieved_GBps": round(n_pairs * yb / (yms * 1e-3) / 1e9, 1)}
        del oy
    stats_out = {k: st[k] for k in ("pairs_rescored", "pairs_full_fp64", "groups_exact", "max_surface_err",
                                    "max_peak_err_sqrt", "tie_band_mixed", "pairs_screened", "pairs_survived",
                                    "check_pairs", "check_changed", "check_peak_err_sqrt", "check_band_frac")}
    # edge track: pairs per second of its alignment stage; algorithmic bytes are
    # the two clips' polygon box tables (64 boxes x 8 bytes each), mostly served
    # from the caches (the kernel is bound by instruction issue)
    edge = None
    if not args.no_edge and stage_t.get("align_edge"):
        e_pairs = tot_e / args.steps
        e_s = stage_t["align_edge"] / args.steps
        edge = {"pairs_per_step": int(e_pairs), "stage_ms": round(e_s * 1e3, 2),
                "pairs_per_s": round(e_pairs / e_s, 1), "alg_bytes_per_pair": 2 * 64 * 8,
                "achieved_GBps": round(e_pairs * 2 * 64 * 8 / e_s / 1e9, 1)}
    stage_ms = {k: round(v * 1000.0 / args.steps, 2) for k, v in stage_t.items()}

    graph = graph_bench(ctx, h, rep, mem)
    contour_obj = None
    if not args.no_contour and not args.no_edge:
        contour_obj = contour_bench(ctx, make_clips, timed, stage_t, args.steps)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cs, rep.cpu().numpy(), mem.cpu().numpy(), args.cpu_seconds)
    h.close()
    del out, rep, mem, last
    torch.cuda.empty_cache()
    mixed_sizes = None if args.no_mixed_sizes else mixed_sizes_bench(ctx)
    torch.cuda.empty_cache()
    schedules = None if args.no_schedule_study else schedule_study(ctx)
    torch.cuda.empty_cache()
    serving = None if args.no_serving else serve_bench(ctx, args.serve_library, args.serve_seconds)

    line = {
        "metric": "aligned pairs/s at 128x128 +-16px (mixed-prec batched vs plain FP32); p99 latency",
        "value": round(value, 1), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": {"mixed": "f16/f32+f64", "fp32": "f32+f64",
                                                          "fp64": "f64"}[args.path],
        "data": "synthetic",
        "config": {"workload": "c128: 50k clips 128x128, 1k templates of 6-24 rects, jitter 4, window +-16, "
                               "cosine 19/20 + edge 3px", "clips": cs.n, "path": args.path,
                   "cosine_pairs_per_step": n_pairs, "edge_pairs_per_step": tot_e // max(args.steps, 1)},
        "roofline": roofline,
        "hbm_read_probe": read_probe,
        "cpu_baseline": cpu,
        "kernel_pairs_per_s": kernel_rate,
        "plain_fp32": comparator,
        "exact_objective": xcorr,
        "xy_separation": xysep,
        "edge": edge,
        "edge_contour": contour_obj,
        "mixed_sizes": mixed_sizes,
        "schedule_study": schedules,
        "stage_ms": stage_ms,
        "stats": stats_out,
        "serving": serving,
        "graph": graph,
    }
    print(json.dumps(line))


def contour_bench(ctx, make_clips, timed, stage_t, steps, t_edge=3, reps=3):
    """Edge track over full boundary edges on the step's clips: contour
    tracing (clip set with CA_CLIPS_CONTOURS against one without), candidate
    generation with the topological-hash test against box sizes alone, and
    the alignment of the surviving pairs, set against the box track's cover."""
    import time

    import torch

    def dirs(b):
        return int((b & 1).sum().item() + ((b >> 1) & 1).sum().item())

    t_plain, t_cont = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        h0 = make_clips()
        torch.cuda.synchronize()
        t_plain.append(time.perf_counter() - t)
        h0.close()
        t = time.perf_counter()
        hc = make_clips(contours=True)
        torch.cuda.synchronize()
        t_cont.append(time.perf_counter() - t)
        if _ < reps - 1:
            hc.close()
    rep_b, mem_b = ctx.prune(hc, "edge", t_edge)
    ob = ctx.align_pairs(hc, rep_b, mem_b, "edge", t_edge)
    # the first call runs the bounds pass (later calls with the same
    # constraint reuse its survivor mask)
    torch.cuda.synchronize()
    t = time.perf_counter()
    rep_c, mem_c = ctx.prune(hc, "contour", t_edge)
    torch.cuda.synchronize()
    prune_s = time.perf_counter() - t
    ctx.align_pairs(hc, rep_c, mem_c, "contour", t_edge)  # warm
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        oc = ctx.align_pairs(hc, rep_c, mem_c, "contour", t_edge)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    al_s = min(ts)
    # the box track on the same (hash-filtered) pairs, for the overlap of the covers
    ob2 = ctx.align_pairs(hc, rep_c, mem_c, "edge", t_edge)
    n_c = rep_c.numel()
    out = {"t_edge_px": t_edge, "clips": int(hc.n),
           "trace_ms": round((min(t_cont) - min(t_plain)) * 1e3, 2),
           "clip_set_ms_without_contours": round(min(t_plain) * 1e3, 2),
           "prune_ms": round(prune_s * 1e3, 2), "pairs": int(n_c), "pairs_box_sizes_only": int(rep_b.numel()),
           "align_ms": round(al_s * 1e3, 2), "pairs_per_s": round(n_c / al_s, 1) if al_s > 0 else None,
           "covering_directions": dirs(oc["bits"]), "covering_directions_box_track": dirs(ob["bits"]),
           "covering_both": dirs(oc["bits"] & ob2["bits"]),
           "no_edge_correspondence_directions": int(((oc["flags"] & (1 << 3)) != 0).sum().item() +
                                                    ((oc["flags"] & (1 << 4)) != 0).sum().item())}
    hc.close()
    return out


def scale_clusters(tracks=("cosine", "contour", "edge")):
    """The method end to end on the 2,000,000-clip workload (128 x 128,
    template densities 0.1-0.6, window +-16) on one GPU: the cosine track at
    19/20 and the edge track over full boundary edges at 2 px with K = 3, and
    the box edge track at 2 px with K = 1 (its K = 3 schedule starts from
    4.0e10 candidates at 4 px, whose relation does not fit one GPU).  Each
    track runs as printed steps: the cover relation at the loosest threshold
    built and sized (the bounds pass, in anchor chunks where its candidate
    mask does not fit, counting and writing the candidates in one sweep, and
    their alignment and compaction), then the loop on it with the
    verification of every member at its center."""
    import ctypes as C

    import numpy as np
    import torch

    import clipgen
    import paper_2512_13133_amd as ca

    cs = clipgen.dense()
    ctx = ca.Context(0)
    t = time.perf_counter()
    h = ctx.clips(cs, fp64=False, contours=True)
    torch.cuda.synchronize()
    out = {"workload": "dense: 2,000,000 clips 128x128, 20,000 templates, densities 0.1-0.6, window +-16",
           "clip_set_s": round(time.perf_counter() - t, 2)}
    log(f"[scale] clip set with contours: {out['clip_set_s']} s")
    runs = {"cosine": ((19, 20), (93, 100), 3), "contour": (2, 4, 3), "edge": (2, 2, 1)}
    for kind in tracks:
        thr, loose, K = runs[kind]
        con = ca.constraint(kind, loose)
        z = C.c_int64(0)
        ctx.reset_stats()
        t = time.perf_counter()
        ctx._check(ctx.lib.ca_cover(ctx.h, ctx._stream(), h.handle, C.byref(con), ca.PATHS["mixed"], 0, None, None,
                                    None, None, None, C.byref(z)))
        torch.cuda.synchronize()
        cover_s = time.perf_counter() - t
        st = ctx.stats()
        cand, screened = st["pairs_survived"], st["pairs_screened"]
        log(f"[scale] {kind}: {cand} candidates of {screened} at the loosest threshold, cover relation of "
            f"{z.value} entries, in {cover_s:.1f} s")
        ctx.reset_stats()
        t = time.perf_counter()
        g = ctx.cluster(h, kind, thr, iterations=K)
        torch.cuda.synchronize()
        st = ctx.stats()
        cl_s = time.perf_counter() - t
        members = int((g["rep_of"] != np.arange(cs.n)).sum())
        out[kind] = {"threshold": list(thr) if isinstance(thr, tuple) else thr, "K": K,
                     "candidates_loosest": int(cand), "pairs_screened": int(screened),
                     "cover_entries_loosest": int(z.value),
                     "cover_s": round(cover_s, 1), "cluster_s": round(cl_s, 1),
                     "clusters": int(g["n_clusters"]), "members": members,
                     "members_verified": int(st["members_verified"]), "center_violations": int(st["center_violations"])}
        log(f"[scale] {kind}: {g['n_clusters']} clusters in {cl_s:.1f} s, {st['center_violations']} violations")
    h.close()
    return out


def mixed_sizes_bench(ctx):
    """The mixed-size workload: 200,000 clips (64, 128, 256 in ratio 4:3:1),
    half-windows 4..32, Zipf(1.2) candidate lists (41.3M directed pairs),
    cosine 97/100, one CA_PATH_AUTO call over the whole list: first with an
    empty tuning table (every bucket tuned on its own pairs), then tuned.  The
    batched MFMA kernels' time and algorithmic bytes (member spectrum and bits
    per pair) come from the library's events."""
    import numpy as np
    import torch

    import clipgen
    t0 = time.time()
    cs, rep, mem = clipgen.mixed()
    log(f"[mixed] generated {cs.n} clips, {rep.size} pairs in {time.time() - t0:.1f}s")
    h = ctx.clips(cs, fp32=True)
    d_rep = torch.from_numpy(rep.astype(np.int32)).cuda()
    d_mem = torch.from_numpy(mem.astype(np.int32)).cuda()
    ctx.autotune_clear()
    times = []
    for it in range(3):
        ctx.reset_stats()
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = ctx.align_pairs(h, d_rep, d_mem, "cosine", (97, 100), "auto")
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        del out
    st = ctx.stats()
    report = ctx.autotune_report()
    h.close()
    by_size = {}
    for N in (64, 128, 256):
        by_size[N] = int((cs.raster_n[rep] == N).sum())
    kernel_gbs = st["main_alg_bytes"] / (st["t_main_ms"] * 1e-3) / 1e9
    return {"workload": "200k clips 64/128/256 (4:3:1), windows 4..32, Zipf(1.2) lists, cosine 97/100",
            "pairs": int(rep.size), "pairs_by_size": by_size,
            "first_call_s": round(times[0], 3), "tuned_call_s": round(min(times[1:]), 3),
            "pairs_per_s": round(rep.size / min(times[1:]), 1),
            "mfma_kernels_ms": round(st["t_main_ms"], 1), "mfma_kernel_launches": st["n_main_launch"],
            "mfma_alg_GBps": round(kernel_gbs, 1), "mfma_hbm_frac": round(kernel_gbs / HBM_PEAK_GBS, 4),
            "rescored": st["pairs_rescored"], "full_fp64": st["pairs_full_fp64"],
            "check_pairs": st["check_pairs"], "check_changed": st["check_changed"],
            "check_band_frac": round(st["check_band_frac"], 4),
            "tuned_paths": [ln.split(" us_per_kpair")[0] for ln in report.splitlines() if ln]}


def schedule_study(ctx):
    """Clusters of the coarse-to-fine loop under different relaxation
    schedules (Sec. 3.1: relaxed coarse stages, strict last stage) on the
    128 x 128 workload at 1:10 (5,000 clips, 100 templates): cosine 19/20 with
    K iterations and total relaxation R, edge 3 px with K iterations and a
    relaxation step in pixels; each entry is one full ca_cluster_schedule call
    (cover at the loosest threshold, set cover, loop, center verification)."""
    import torch

    import clipgen
    cs = clipgen.c128(n_clips=5000, n_templates=100)
    h = ctx.clips(cs, fp32=True)
    out = {"workload": "c128 at 1:10: 5,000 clips, 100 templates", "cosine": [], "edge": []}
    runs = [("cosine", (19, 20), 1, (0, 1))] + [("cosine", (19, 20), K, (r, 100)) for K in (2, 3, 4)
                                                for r in (1, 2, 4)]
    runs += [("edge", 3, 1, 0)] + [("edge", 3, K, st) for K in (2, 3) for st in (1, 2)]
    for kind, thr, K, relax in runs:
        torch.cuda.synchronize()
        t = time.perf_counter()
        got = ctx.cluster(h, kind, thr, iterations=K, relax=relax)
        ms = (time.perf_counter() - t) * 1e3
        entry = {"K": K, "clusters": got["n_clusters"], "ms": round(ms, 1)}
        entry["relax"] = f"{relax[0]}/{relax[1]}" if kind == "cosine" else f"{relax} px/step"
        out[kind].append(entry)
    h.close()
    return out


def graph_bench(ctx, h, rep, mem, n=4096, reps=50):
    """Small batches: the mixed alignment of n pairs as one captured graph
    launch against the eager call (launches plus its host round trips)."""
    import torch
    r, m = rep[:n].clone(), mem[:n].clone()
    g = ctx.graph(h, n, (19, 20))
    g.set_pairs(r, m)
    for _ in range(3):
        g.launch()
        ctx.align_pairs(h, r, m, "cosine", (19, 20), "mixed")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.launch()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.align_pairs(h, r, m, "cosine", (19, 20), "mixed")
    torch.cuda.synchronize()
    t_eager = (time.perf_counter() - t0) / reps
    same = all(bool(torch.equal(g.out[k], v)) for k, v in
               ctx.align_pairs(h, r, m, "cosine", (19, 20), "mixed").items() if k != "flags")
    g.close()
    return {"pairs": n, "graph_ms": round(t_graph * 1e3, 3), "eager_ms": round(t_eager * 1e3, 3),
            "identical_results": same}


def serve_bench(ctx, n_library, seconds, slots=4):
    """Serving: a device-resident library of 128 x 128 representatives (one per
    template); request batches of log-normal size (median 64, sigma 1, at most
    10,000 clips) drawn from library templates with jitter 4 and offsets +-16,
    arriving as a Poisson stream.  First the saturation rate with a full queue,
    then latency at half of it and at 80% of it."""
    import threading

    import numpy as np

    import clipgen
    import paper_2512_13133_amd as ca
    t0 = time.time()
    lib, _, tpl = clipgen.serving(n_library=n_library, n_requests=0, return_templates=True)
    rng = np.random.default_rng(2026)

    def make_request():
        size = int(np.clip(np.rint(rng.lognormal(np.log(64), 1.0)), 1, 10_000))
        return clipgen.make_clips(rng, tpl, 128, size, 4, 16)

    hlib = ctx.clips(lib, fp32=True)
    srv = ca.Server(ctx, hlib, (19, 20), slots=slots, hbm_budget_bytes=64 << 30)
    log(f"[serve] library {lib.n} ready in {time.time() - t0:.1f}s")

    def run(trace, pace):
        """Submit (arrival_s, ClipSet) requests; return per-request latency (s) and wall time."""
        lat = [None] * len(trace)
        pending = {}
        lock = threading.Lock()
        finished = threading.Event()
        start = time.perf_counter()

        def collector():
            while True:
                with lock:
                    items = list(pending.items())
                for idx, (rid, n, arr) in items:
                    if srv.poll(rid, n) is not None:
                        lat[idx] = time.perf_counter() - start - arr
                        with lock:
                            del pending[idx]
                if finished.is_set():
                    with lock:
                        if not pending:
                            return
                time.sleep(0.0003)

        th = threading.Thread(target=collector)
        th.start()
        for idx, (arr, req) in enumerate(trace):
            if pace:
                delay = arr - (time.perf_counter() - start)
                if delay > 0:
                    time.sleep(delay)
            else:
                arr = time.perf_counter() - start
            while True:
                try:
                    rid = srv.submit(req)
                    break
                except ca.ClipAlignError as e:
                    if e.status != ca.CA_EBUSY:
                        raise
                    time.sleep(0.0005)
            with lock:
                pending[idx] = (rid, req.n, arr)
        finished.set()
        th.join()
        return np.array(lat), time.perf_counter() - start

    # saturation: everything queued at once
    warm = [(0.0, make_request()) for _ in range(8)]
    run(warm, False)
    sat_trace = [(0.0, make_request()) for _ in range(120)]
    st0 = srv.stats()
    lat_sat, wall_sat = run(sat_trace, False)
    st1 = srv.stats()
    sat_qps = len(sat_trace) / wall_sat
    qps = 0.5 * sat_qps
    n_req = max(20, int(qps * seconds))
    arrivals = np.cumsum(rng.exponential(1.0 / qps, size=n_req))
    trace = [(float(a), make_request()) for a in arrivals]
    lat, wall = run(trace, True)
    st2 = srv.stats()
    # and at 80% of saturation
    qps80 = 0.8 * sat_qps
    n80 = max(20, int(qps80 * seconds))
    arr80 = np.cumsum(rng.exponential(1.0 / qps80, size=n80))
    lat80, wall80 = run([(float(a), make_request()) for a in arr80], True)
    srv.close()
    hlib.close()
    clips = sum(r.n for _, r in trace)
    return {"library": lib.n, "slots": slots, "saturation_qps": round(sat_qps, 1),
            "saturation_pairs_per_s": round((st1["candidate_pairs"] - st0["candidate_pairs"]) / wall_sat, 1),
            "qps_target": round(qps, 1), "qps_achieved": round(n_req / wall, 1), "requests": n_req,
            "clips": clips, "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
            "pairs_per_s": round((st2["candidate_pairs"] - st1["candidate_pairs"]) / wall, 1),
            "at_80pct": {"qps_target": round(qps80, 1), "qps_achieved": round(n80 / wall80, 1), "requests": n80,
                         "p50_ms": round(float(np.percentile(lat80, 50)) * 1e3, 2),
                         "p99_ms": round(float(np.percentile(lat80, 99)) * 1e3, 2)},
            "request_sizes": "round(LogNormal(ln 64, 1)) clipped to [1, 10000]"}


def copy_probe(nbytes, reps=3):
    """A plain device-to-device copy of known size: its FETCH_SIZE / WRITE_SIZE
    counters calibrate the traffic figures of the roofline."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    src.sum()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    t = time.perf_counter()
    for _ in range(reps):
        src.sum()
    torch.cuda.synchronize()
    dt_sum = (time.perf_counter() - t) / reps
    import paper_2512_13133_amd as ca
    ms_read = ca.probe_read_bandwidth(src, reps=10)
    print(json.dumps({"copy_bytes": src.numel() * 4, "reps": reps, "ms": dt * 1e3,
                      "GBps_read_plus_write": 2 * src.numel() * 4 / dt / 1e9,
                      "sum_ms": dt_sum * 1e3, "GBps_read_only_sum": src.numel() * 4 / dt_sum / 1e9,
                      "read_probe_ms": ms_read, "GBps_read_probe": src.numel() * 4 / (ms_read * 1e-3) / 1e9}))


def _cpu_worker(args):
    import numpy as np

    from oracle import cover
    cs, rep, mem = args
    t = time.perf_counter()
    cover.align_pairs_cosine(cs, rep, mem, 19, 20, workers=1)
    return rep.size, time.perf_counter() - t


def cpu_baseline(cs, rep, mem, seconds):
    """The FP64 oracle on a bounded sample of the same cosine pairs, all host cores."""
    import multiprocessing as mp

    import numpy as np
    # one GPU's share of the host: 16 cores (the host may show more; worker
    # pools beyond one GPU's share are not run)
    visible = len(os.sched_getaffinity(0))
    cores = max(1, min(visible, 16))
    # size the sample from a short single-core probe
    rng = np.random.default_rng(1234)
    probe = rng.choice(rep.size, size=min(200, rep.size), replace=False)
    n, dt = _cpu_worker((cs, rep[probe], mem[probe]))
    per_core = n / dt
    total = int(min(rep.size, per_core * cores * seconds))
    pick = np.sort(rng.choice(rep.size, size=max(total, cores), replace=False))
    chunks = np.array_split(pick, cores)
    ctx = mp.get_context("fork")
    t = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_cpu_worker, [(cs, rep[c], mem[c]) for c in chunks])
    wall = time.perf_counter() - t
    done = sum(r[0] for r in res)
    return {"value": round(done / wall, 1), "unit": "pairs/s", "cores": cores, "cores_visible": visible,
            "per_core": round(done / wall / cores, 1), "kind": "oracle",
            "sample": f"{done} cosine candidate pairs of the timed step, uniform sample, FP64 numpy oracle, "
                      f"both directions per pair"}


if __name__ == "__main__":
    main()
