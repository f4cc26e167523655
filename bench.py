#!/usr/bin/env python3
"""Benchmark of the multi-receiver Gaussian rasterizer on one MI355X.

Metric: receiver-views per second on the 90 x 360 grid for one fused render
of all receivers, beside a per-receiver launch loop (the same library called
once per receiver) on the same GPU, as in the paper's inference comparison
(Table 2; App. G.3).  Workload: 50,000 seeded synthetic Gaussians in a
10 x 10 x 3 m box, 64 receivers, conditioning-MLP radiance, one transmitter.

One step = one pass of the whole hot path over all receivers: projection,
per-view depth sort, binning, pair sort, MLP radiance, compositing and the
power reduction.  Inputs are resident in HBM before the timed region.

Prints one JSON line.  Per-stage times come from HIP events recorded by the
library on the launch stream during a second, profiled pass of the same
steps; the roofline entry is for the stage with the largest share.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

METRIC = "receiver-views/s (90x360 grid) multi-rx fused vs per-rx loop; serve p50/p99"

# MI355X published peaks and the derived vector-ALU rate
PEAK_HBM_GBS = 8000.0
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_FP16_MFMA_TFLOPS = 2500.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane operations per second
# (one FP32 op per lane per cycle; an FMA counts as one operation here)
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
MLP_FLOP_PER_PAIR = 2 * 64 * 64 + 2 * 64 * 2     # layers 2 and 3 per (receiver, visible Gaussian)
MLP_MFMA_FLOP_PER_PAIR = 3 * 2 * 64 * 64         # split FP16: three FP16 products for layer 2
BLEND_OPS_PER_PAIR = 16      # lane-ops per composited (pixel, Gaussian) pair: offsets, quadratic form,
                             # exp (4), clamp and test, transmittance update, one complex accumulate
BLEND_OPS_PER_EXTRA_RX = 2   # TX mode: each further receiver sharing the weight adds one complex FMA
SORT_BYTES_PER_KEY_PASS = 16  # read and write one (u32 key, u32 value) per pass
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "k_blend_fwd1_c1_rx_traffic.txt")
SQ_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "c1_rx_sq_counters.txt")
STATS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "k_blend_fwd1_c1_rx_stats.txt")
VALU_ISSUE_PEAK = 256 * 2.4e9   # wave64 VALU instructions per second (one per CU per cycle)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c1", help="workload preset (c1 = 50k Gaussians, 64 receivers)")
    ap.add_argument("--mode", default="rx", choices=["rx", "tx"],
                    help="rx: each receiver is its own view; tx: receivers share the transmitter's view")
    ap.add_argument("--loop-steps", type=int, default=3)
    ap.add_argument("--no-loop", action="store_true")
    ap.add_argument("--no-other-mode", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target wall time of the oracle sample")
    ap.add_argument("--no-train", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-rxcond", action="store_true", help="skip the paper's conditioned-radiance workloads")
    ap.add_argument("--no-scale", action="store_true", help="skip the 1M-Gaussian scale workload")
    ap.add_argument("--serve-queries", type=int, default=2000, help="measured queries per arrival rate")
    ap.add_argument("--serve-warmup", type=int, default=200, help="warm-up queries before the serving runs")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run a plain copy of this many MiB (counter calibration for profiled runs)")
    return ap.parse_args()


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / max(steps, 1)


def gpu_part(args):
    import torch
    from paper_2605_24290_amd import rxgs
    from paper_2605_24290_amd import scenes as S

    wl = S.make_workload(args.config)
    sc = wl.scene
    dev = torch.device("cuda", 0)
    r = rxgs.Renderer(wl.grid)
    r.upload_scene(sc.means, sc.log_scales, sc.quats, sc.logits, radiance=sc.radiance, features=sc.features)
    if sc.features is not None:
        r.upload_mlp(S.flat_mlp(wl.mlp))
    rx = torch.as_tensor(wl.rx, device=dev)
    tx = torch.as_tensor(wl.tx, device=dev)
    N = rx.shape[0]
    H, W = wl.grid.H, wl.grid.W
    C = torch.empty((N, 2, H, W), device=dev)
    P = torch.empty((N,), device=dev)

    def fused(mode):
        return lambda: r.render(rx, tx=tx, mode=mode, out=(C, P))

    def loop(mode):
        def f():
            for j in range(N):
                r.render(rx[j:j + 1], tx=tx, mode=mode, out=(C[j:j + 1], P[j:j + 1]))
        return f

    res = {}
    modes = [args.mode] + ([] if args.no_other_mode else [m for m in ("rx", "tx") if m != args.mode])
    for mode in modes:
        ms = timed(fused(mode), args.steps, args.warmup)
        entry = {"ms_per_step": ms, "rx_views_per_s": N * 1000.0 / ms}
        # profiled pass: per-stage event times over the same number of steps
        r.profile(True)
        r.profile_read(reset=True)
        r.profile_counts(reset=True)
        ms_prof = timed(fused(mode), args.steps, 0)
        stages = r.profile_read(reset=True)
        counts = r.profile_counts(reset=True)
        r.profile(False)
        entry["ms_per_step_profiled"] = ms_prof
        entry["stages_ms_per_step"] = {k: v[1] / args.steps for k, v in stages.items()}
        entry["stage_launches"] = {k: v[0] for k, v in stages.items()}
        # MLP work the pair kernels evaluated, counted on the device per render
        entry["mlp_evaluated"] = {k: v / args.steps for k, v in counts.items()}
        # sizes of one render (visible Gaussians per view, pairs)
        saved = rxgs.Saved(r)
        r.render(rx, tx=tx, mode=mode, saved=saved, out=(C, P))
        torch.cuda.synchronize()
        info = saved.info()
        nvis = saved.export(rxgs.EXPORT_NVIS, "int32", (info["V"],))
        pairs_mlp = int(nvis.sum()) if mode == "rx" else int(nvis[0]) * N
        rpc = 1 if mode == "rx" else min(16, 1 << max(0, (N - 1).bit_length()))
        entry["sizes"] = {"views": info["V"], "visible_total": int(nvis.sum()), "tile_pairs": info["D"],
                          "mlp_pairs": pairs_mlp, "sort_keys": info["V"] * info["K_pad"],
                          "composited": info["n_composited"], "composited_px": info["n_composited_px"],
                          "evaluated_px": info["n_evaluated_px"], "walked_px": info["n_walked_px"],
                          "chunks_per_view": 1 if mode == "rx" else -(-N // rpc)}
        saved.close()
        if mode == args.mode and sc.features is not None:
            entry["mlp_fp32"] = mlp_fp32_timing(args, wl, rx, tx, C, P, mode)
        if not args.no_loop:
            ms_loop = timed(loop(mode), args.loop_steps, 1)
            entry["per_rx_loop"] = {"ms_per_step": ms_loop, "rx_views_per_s": N * 1000.0 / ms_loop,
                                    "fused_speedup": ms_loop / ms}
        res[mode] = entry
    r.close()
    return wl, res


def mlp_fp32_timing(args, wl, rx, tx, C, P, mode):
    """The same render with the pair MLP on FP32 matrix cores throughout
    (RXGS_MLP_FP32=1 at the MLP upload) instead of split FP16."""
    from paper_2605_24290_amd import rxgs
    from paper_2605_24290_amd import scenes as S
    sc = wl.scene
    r = rxgs.Renderer(wl.grid)
    r.upload_scene(sc.means, sc.log_scales, sc.quats, sc.logits, features=sc.features)
    old = os.environ.get("RXGS_MLP_FP32")
    os.environ["RXGS_MLP_FP32"] = "1"
    try:
        r.upload_mlp(S.flat_mlp(wl.mlp))
    finally:
        if old is None:
            del os.environ["RXGS_MLP_FP32"]
        else:
            os.environ["RXGS_MLP_FP32"] = old
    f = lambda: r.render(rx, tx=tx, mode=mode, out=(C, P))
    ms = timed(f, args.steps, args.warmup)
    r.profile(True)
    r.profile_read(reset=True)
    timed(f, args.steps, 0)
    stages = r.profile_read(reset=True)
    r.profile(False)
    r.close()
    st = {k: v[1] / args.steps for k, v in stages.items()}
    return {"ms_per_step": ms, "rx_views_per_s": rx.shape[0] * 1000.0 / ms,
            "mlp_pairs_ms": st.get("mlp_pairs", 0.0) + st.get("mlp_far", 0.0)}


def train_step_part(args):
    """Forward + L2 loss gradient + hand-written backward on the 100k-Gaussian,
    32-receiver workload (gradients for every scene and MLP parameter; no
    optimizer update)."""
    import torch
    from paper_2605_24290_amd import rxgs
    from paper_2605_24290_amd import scenes as S

    wl = S.make_workload("c2")
    sc = wl.scene
    dev = torch.device("cuda", 0)
    r = rxgs.Renderer(wl.grid)
    r.upload_scene(sc.means, sc.log_scales, sc.quats, sc.logits, features=sc.features)
    r.upload_mlp(S.flat_mlp(wl.mlp))
    rx = torch.as_tensor(wl.rx, device=dev)
    tx = torch.as_tensor(wl.tx, device=dev)
    Y = torch.as_tensor(wl.targets, device=dev)
    saved = rxgs.Saved(r)
    grads = None
    out = {}
    for mode in ("rx", "tx"):
        def step():
            nonlocal grads
            C, P, _ = r.render(rx, tx=tx, mode=mode, saved=saved)
            grads = r.backward(saved, C, 2.0 * (C - Y), None, grads)
        ms = timed(step, max(3, args.steps // 4), 2)
        r.profile(True)
        r.profile_read(reset=True)
        timed(step, 3, 0)
        stages = r.profile_read(reset=True)
        r.profile(False)
        out[mode] = {"ms_per_step": ms, "rx_views_per_s": wl.rx.shape[0] * 1000.0 / ms,
                     "stages_ms_per_step": {k: v[1] / 3 for k, v in stages.items()}}
        # the same step with the fixed-order (bitwise-repeatable) backward
        r.deterministic(True)
        ms_det = timed(step, max(3, args.steps // 4), 2)
        r.profile(True)
        r.profile_read(reset=True)
        timed(step, 3, 0)
        stages = r.profile_read(reset=True)
        r.profile(False)
        r.deterministic(False)
        out[mode]["deterministic"] = {"ms_per_step": ms_det, "vs_atomic": ms_det / ms,
                                      "stages_ms_per_step": {k: v[1] / 3 for k, v in stages.items()}}
    saved.close()
    r.close()
    return {"workload": f"c2: {sc.K} Gaussians, {wl.rx.shape[0]} receivers, 90x360, MLP, L2 loss, forward + "
                        "backward to all parameters (no optimizer update)", **out}


def scale_part(args):
    """The 1M-Gaussian scale workload: the training step over 512 RX views, and
    a 4,096-receiver coverage map of one transmitter streamed in receiver
    chunks sized to half the free HBM."""
    import torch
    from paper_2605_24290_amd import rxgs
    from paper_2605_24290_amd import scenes as S

    dev = torch.device("cuda", 0)
    out = {}
    wl = S.make_workload("c4")
    sc = wl.scene
    r = rxgs.Renderer(wl.grid)
    r.upload_scene(sc.means, sc.log_scales, sc.quats, sc.logits, features=sc.features)
    r.upload_mlp(S.flat_mlp(wl.mlp))
    rx = torch.as_tensor(wl.rx, device=dev)
    Y = torch.as_tensor(wl.targets, device=dev)
    saved = rxgs.Saved(r)
    grads = None

    def step():
        nonlocal grads
        C, P, _ = r.render(rx, mode="rx", saved=saved)
        grads = r.backward(saved, C, 2.0 * (C - Y), None, grads)
    ms = timed(step, 2, 1)
    info = saved.info()
    out["train_step_rx"] = {"ms_per_step": ms, "rx_views_per_s": wl.rx.shape[0] * 1000.0 / ms,
                            "tile_pairs": int(info["D"]), "visible": int(info["n_visible"])}
    saved.close()
    r.close()
    del Y, rx, grads
    torch.cuda.empty_cache()

    wl = S.make_workload("c4", N=4096, targets=False)
    sc = wl.scene
    r = rxgs.Renderer(wl.grid)
    r.upload_scene(sc.means, sc.log_scales, sc.quats, sc.logits, features=sc.features)
    r.upload_mlp(S.flat_mlp(wl.mlp))
    rx = torch.as_tensor(wl.rx, device=dev)
    tx = torch.as_tensor(wl.tx, device=dev)
    N = wl.rx.shape[0]
    C = torch.empty((N, 2, wl.grid.H, wl.grid.W), device=dev)
    P = torch.empty((N,), device=dev)
    nch = [0]

    def cover():
        nch[0] = r.render_chunked(rx, tx=tx, mode="tx", out=(C, P))[2]
    ms = timed(cover, 3, 1)
    out["coverage_tx"] = {"ms_per_map": ms, "rx_views_per_s": N * 1000.0 / ms, "chunks": nch[0]}
    r.close()
    del C, P
    torch.cuda.empty_cache()
    return {"workload": f"c4: {sc.K} Gaussians in a 40x40x4 m box, 90x360, MLP; training step over 512 RX views "
                        f"(L2 loss, all gradients); coverage map of {N} receivers of one transmitter", **out}


def rxcond_part(args):
    """The paper's own radiance path (FiLM global branch, occupancy local
    branch, FLE / SH basis) on its inference shape: 32,000 Gaussians in an
    8 x 6 x 3 m room, 21 receivers, 90 x 360, one transmitter (Table 2's
    setting; App. E Table 4: lmax 9, F = 6, d = 64, S = 16, 128^3 grid).
    Fused render of all receivers against the same library called once per
    receiver; both view modes; the SH backbone (degree 4) and a 26-channel
    CSI-shaped signal on a 72 x 18 grid beside it."""
    import torch
    from paper_2605_24290_amd import rxgs
    from paper_2605_24290_amd import scenes as S

    dev = torch.device("cuda", 0)
    out = {}
    cases = [("fle_l9", S.BASIS_FLE, 9, 1, None), ("sh_l4", S.BASIS_SH, 4, 1, None),
             ("csi_c26_fle_l4", S.BASIS_FLE, 4, 26, S.Grid(18, 72, 0.0, math.radians(5.0)))]
    for name, kind, lmax, C, grid in cases:
        wl = S.make_workload("paper", grid=grid, use_mlp=False)
        sc = wl.scene
        m = S.make_rxcond_model(sc.K, kind=kind, lmax=lmax, C=C, F=6, H=64)
        r = rxgs.Renderer(wl.grid)
        r.upload_scene(sc.means, sc.log_scales, sc.quats, sc.logits)
        t0 = time.perf_counter()
        r.upload_rxcond(m)
        torch.cuda.synchronize()
        t_up = time.perf_counter() - t0
        rx = torch.as_tensor(wl.rx, device=dev)
        tx = torch.as_tensor(wl.tx, device=dev)
        N = rx.shape[0]
        entry = {"gaussians": sc.K, "receivers": N, "channels": C, "basis": "FLE" if kind == S.BASIS_FLE else "SH",
                 "lmax": lmax, "components": (lmax + 1) ** 2, "grid": [wl.grid.H, wl.grid.W],
                 "upload_s": t_up}
        for mode in ("tx", "rx"):
            ms = timed(lambda: r.render_rxcond(rx, tx=tx, mode=mode), args.steps, args.warmup)
            r.profile(True)
            r.profile_read(reset=True)
            timed(lambda: r.render_rxcond(rx, tx=tx, mode=mode), 3, 0)
            stages = r.profile_read(reset=True)
            r.profile(False)

            def loop():
                for j in range(N):
                    r.render_rxcond(rx[j:j + 1], tx=tx, mode=mode)
            ms_loop = timed(loop, 2, 1)
            entry[mode] = {"ms_per_render": ms, "rx_views_per_s": N * C * 1000.0 / ms,
                           "per_rx_loop_ms": ms_loop, "fused_speedup": ms_loop / ms,
                           "stages_ms_per_render": {k: v[1] / 3 for k, v in stages.items()}}
        r.close()
        out[name] = entry
        torch.cuda.empty_cache()
    return {"workload": "paper inference shape: 32,000 Gaussians (8 x 6 x 3 m), 21 receivers, 1 transmitter; "
                        "the paper's conditioned radiance; rx_views_per_s counts (receiver, channel) spectra",
            "paper_h100_ms_all_21_rx": {"GSRF (FLE)": 31.2, "RF-3DGS (SH)": 35.3}, **out}


def serving_part(args):
    """Continuous batching on the 200k-Gaussian scene: saturation throughput of
    a burst, then open-loop Poisson arrivals at 0.3 / 0.6 / 0.9 of it."""
    from paper_2605_24290_amd import rxgs, serving
    from paper_2605_24290_amd import scenes as S

    wl = S.make_workload("c3", N=1)
    sc = wl.scene
    r = rxgs.Renderer(wl.grid)
    r.upload_scene(sc.means, sc.log_scales, sc.quats, sc.logits, features=sc.features)
    r.upload_mlp(S.flat_mlp(wl.mlp))
    box = S.PRESETS["c3"].box
    srv = rxgs.Server(r, mode="tx", slots=2, max_rx_per_batch=4096, max_queries_per_batch=64)
    warm = S.serving_queries(1, args.serve_warmup, box)
    serving.run_burst(srv, warm)
    qs = S.serving_queries(S.BASE_SEED + 3000, args.serve_queries, box)
    sat = serving.run_burst(srv, qs)
    rates = {}
    for f in (0.3, 0.6, 0.9):
        rates[str(f)] = serving.run_open_loop(srv, qs, rate=f * sat["achieved_qps"])
    st = srv.stats()
    srv.stop()
    r.close()
    return {"workload": f"c3: {sc.K} Gaussians resident, TX mode, queries of 1-256 receivers (log-uniform), "
                        f"{args.serve_warmup} warm-up queries, then {args.serve_queries} queries per rate, 2 slots",
            "saturation": sat,
            "rates_x_saturation": rates, "server_stats": st}


# the sources the forward kernels are compiled from (host-only files excluded)
KERNEL_SOURCES = ("device_common.h", "kernels.hip", "rxgs_internal.h")


def source_digest() -> str:
    """SHA-256 of the forward kernels' sources, to tell whether stored counter
    readings still describe the kernels that were just timed."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2605_24290_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()


def stored_figure(path: str, field: str, kernel: str, workload: str):
    """A per-launch figure of `kernel` from a committed rocprofv3 summary; None
    if there is none for this kernel and workload or the sources changed since."""
    try:
        with open(path) as fh:
            kv = dict(line.split(":", 1) for line in fh
                      if ":" in line and not line.startswith("#") and not line.startswith(" "))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel") != kernel or kv.get("workload") != workload or kv.get("source_sha256") != source_digest():
        return None
    try:
        return float(kv[field])
    except (KeyError, ValueError):
        return None


def stored_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE summary, scaled by
    the copy-kernel calibration it records."""
    return stored_figure(TRAFFIC_FILE, "hbm_bytes_per_launch", kernel, workload)


def roofline_for(entry, mode, workload, K=0):
    """Roofline entry of the stage with the largest time share; the time is the
    stage's average from HIP events the library records on the launch stream."""
    st = entry["stages_ms_per_step"]
    top = max(st, key=st.get)
    t_s = st[top] / 1000.0
    sz = entry["sizes"]
    if top == "blend_fwd":
        if mode == "rx":
            ops = BLEND_OPS_PER_PAIR * sz["composited"]
        else:   # weights once per view pixel, one complex FMA per further receiver
            per_view = sz["composited_px"] / max(sz["chunks_per_view"], 1)
            ops = BLEND_OPS_PER_PAIR * per_view + BLEND_OPS_PER_EXTRA_RX * (sz["composited"] - per_view)
        ach = ops / t_s / 1e12
        # executed wave64 VALU instructions per launch (SQ_INSTS_VALU of the
        # committed counter run) against the issue peak, over the live launch time
        insts = stored_figure(SQ_FILE, "valu_wave_insts_per_launch", "k_blend_fwd1", workload)
        # the same work over the kernel's average duration in the committed
        # rocprofv3 --kernel-trace --stats summary (None once the sources changed)
        avg_ns = stored_figure(STATS_FILE, "avg_ns_per_launch", "k_blend_fwd1", workload)
        frac_rp = None if not avg_ns else ops / (avg_ns * 1e-9) / 1e12 / PEAK_VALU_TOPS
        return {"kernel": "k_blend_fwd1", "bound": "alu", "achieved": ach, "peak": PEAK_VALU_TOPS,
                "unit": "Tops/s", "frac": ach / PEAK_VALU_TOPS, "frac_rocprof": frac_rp,
                "rocprof_avg_us": None if not avg_ns else avg_ns / 1000.0, "event_avg_us": t_s * 1e6,
                "traffic": stored_traffic("k_blend_fwd1", workload),
                "valu_issue_frac": None if insts is None else insts / (VALU_ISSUE_PEAK * t_s),
                "work": f"{BLEND_OPS_PER_PAIR} lane-ops x {sz['composited']} composited (pixel, Gaussian) pairs"}
    if top == "mlp_pairs":
        flop = MLP_MFMA_FLOP_PER_PAIR * mlp_pairs_evaluated(entry)
        ach = flop / t_s / 1e12
        return {"kernel": "k_mlp_pairs", "bound": "mfma", "achieved": ach, "peak": PEAK_FP16_MFMA_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / PEAK_FP16_MFMA_TFLOPS, "traffic": None,
                "work": f"{MLP_MFMA_FLOP_PER_PAIR} FP16 MFMA FLOP x {mlp_pairs_evaluated(entry)} (receiver, "
                        f"position) pairs evaluated ({MLP_FLOP_PER_PAIR} FP32-equivalent)"}
    # any other stage: its HBM roofline from the per-stage model
    row = stage_rooflines(entry, mode, K)["stages"].get(top, {})
    if row.get("bound") == "hbm":
        ach = row["work"] / t_s / 1e9
        return {"kernel": STAGE_KERNELS.get(top, top), "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": ach / PEAK_HBM_GBS, "traffic": None, "work": row["work_model"]}
    return {"kernel": top, "bound": "unknown", "achieved": None, "peak": None, "unit": None, "frac": None,
            "traffic": None}


# the kernels behind the stage names
STAGE_KERNELS = {"project": "k_gauss_prep + k_keys", "sort_depth": "k_sort_pass (4 passes)",
                 "emit_records": "k_emit1", "emit_pairs": "k_bin_pairs (or k_emit2)", "sort_pairs": "k_sort_pass"}


# Algorithmic work per stage of one render (bytes that must cross HBM, lane-ops,
# matrix FLOP), for the per-stage roofline fractions and the overall one,
# sum of t_roof over the stages / measured time per render.
EMIT_RECORD_BYTES = 84 + 56   # per visible entry: order index + projection terms read; record,
                              # box, index and pair slot written
EMIT_PAIR_BYTES_ENTRY = 20    # per visible entry: box and first pair slot read
PAIR_BYTES = 8                # per pair: tile and sorted position written (emission before a pair sort)
BIN_PAIR_BYTES = 4            # per pair: sorted position written in its tile list (direct binning)
PAIR_SORT_BYTES = 4 + SORT_BYTES_PER_KEY_PASS   # per pair: histogram read + one 8-bit pass


def mlp_pairs_evaluated(entry):
    """(receiver, position) pairs the pair MLP evaluated per render, counted on
    the device in the profiled pass (prefix and far launches together)."""
    ev = entry.get("mlp_evaluated")
    return int(round(ev["mlp_pairs"])) if ev else entry["sizes"]["mlp_pairs"]


def stage_rooflines(entry, mode, K):
    """Per stage: bound, algorithmic work, t_roof = work / peak, the measured
    time (HIP events, per render) and t_roof / t; the overall fraction
    divides the sum of t_roof by the measured time per render."""
    st = entry["stages_ms_per_step"]
    sz = entry["sizes"]
    nvis, D, VK = sz["visible_total"], sz["tile_pairs"], sz["sort_keys"]
    if mode == "rx":
        blend_ops = BLEND_OPS_PER_PAIR * sz["composited"]
    else:
        per_view = sz["composited_px"] / max(sz["chunks_per_view"], 1)
        blend_ops = BLEND_OPS_PER_PAIR * per_view + BLEND_OPS_PER_EXTRA_RX * (sz["composited"] - per_view)
    model = {
        "project": ("hbm", 44 * K + 8 * VK, "44 B per Gaussian read, 8 B per (view, Gaussian) key written"),
        "sort_depth": ("hbm", 4 * SORT_BYTES_PER_KEY_PASS * VK,
                       f"{4 * SORT_BYTES_PER_KEY_PASS} B per (view, Gaussian) key (4 passes)"),
        "emit_records": ("hbm", EMIT_RECORD_BYTES * nvis, f"{EMIT_RECORD_BYTES} B per visible entry"),
        "emit_pairs": (("hbm", EMIT_PAIR_BYTES_ENTRY * nvis + PAIR_BYTES * D,
                        f"{EMIT_PAIR_BYTES_ENTRY} B per visible entry + {PAIR_BYTES} B per pair")
                       if "sort_pairs" in st else
                       ("hbm", EMIT_PAIR_BYTES_ENTRY * nvis + BIN_PAIR_BYTES * D,
                        f"{EMIT_PAIR_BYTES_ENTRY} B per visible entry + {BIN_PAIR_BYTES} B per pair (direct binning)")),
        "sort_pairs": ("hbm", PAIR_SORT_BYTES * D, f"{PAIR_SORT_BYTES} B per pair"),
        "mlp_pairs": ("mfma", MLP_MFMA_FLOP_PER_PAIR * mlp_pairs_evaluated(entry),
                      f"{MLP_MFMA_FLOP_PER_PAIR} FP16 MFMA FLOP per (receiver, position) pair evaluated "
                      "(device count; the far launch's time and pairs included)"),
        "blend_fwd": ("alu", blend_ops, f"{BLEND_OPS_PER_PAIR} lane-ops per composited pair"),
    }
    peak = {"hbm": PEAK_HBM_GBS * 1e9, "mfma": PEAK_FP16_MFMA_TFLOPS * 1e12, "alu": PEAK_VALU_TOPS * 1e12}
    rows, t_roof_sum = {}, 0.0
    st = dict(st)
    if "mlp_far" in st and "mlp_pairs" in st:   # the counted pairs cover both launches
        st["mlp_pairs"] += st.pop("mlp_far")
        rows["mlp_far"] = {"bound": "included in mlp_pairs"}
    for name, t_ms in st.items():
        if name not in model:
            rows[name] = {"bound": "negligible", "t_us": t_ms * 1e3}
            continue
        bound, work, desc = model[name]
        t_roof = work / peak[bound]
        t_roof_sum += t_roof
        rows[name] = {"bound": bound, "work": work, "work_model": desc, "t_roof_us": t_roof * 1e6,
                      "t_us": t_ms * 1e3, "frac": t_roof / (t_ms * 1e-3) if t_ms > 0 else None}
    return {"stages": rows, "overall_frac": t_roof_sum / (entry["ms_per_step"] * 1e-3),
            "note": "stage times from the profiled pass; overall = sum of t_roof / unprofiled time per render"}


def copy_calibration(mib: int):
    """A plain elementwise copy of known size (read mib MiB, write mib MiB),
    for scaling the FETCH_SIZE / WRITE_SIZE counters of a profiled run."""
    import torch
    n = mib * (1 << 20) // 4
    x = torch.ones(n, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(f"copy calibration: {n * 4} bytes read and written per launch", flush=True)


def cpu_baseline(args, wl, mode):
    """The FP64 C oracle on the host, on a bounded sample of the same workload:
    renders of the first n receivers (n sized from a one-receiver calibration),
    repeated until about --cpu-seconds of wall time have passed."""
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from oracle import oracle as O
    threads = len(os.sched_getaffinity(0))
    rx1 = wl.rx[:1]
    cen, rv = O.views_for(mode, wl.tx, rx1)
    t0 = time.perf_counter()
    O.render(wl.scene, wl.grid, cen, rx1, rv, mlp=wl.mlp, nthreads=threads)
    t1 = time.perf_counter() - t0
    n = int(max(1, min(wl.rx.shape[0], math.floor(args.cpu_seconds / max(t1, 1e-3)))))
    rxs = wl.rx[:n]
    cen, rv = O.views_for(mode, wl.tx, rxs)
    views, dt, reps = 0, 0.0, 0
    while reps == 0 or dt < args.cpu_seconds:
        t0 = time.perf_counter()
        O.render(wl.scene, wl.grid, cen, rxs, rv, mlp=wl.mlp, nthreads=threads)
        dt += time.perf_counter() - t0
        views += n
        reps += 1
    # one thread: one receiver, repeated for about a third of the time
    rx1 = wl.rx[:1]
    cen1, rv1 = O.views_for(mode, wl.tx, rx1)
    v1, d1 = 0, 0.0
    while v1 == 0 or d1 < args.cpu_seconds / 3:
        t0 = time.perf_counter()
        O.render(wl.scene, wl.grid, cen1, rx1, rv1, mlp=wl.mlp, nthreads=1)
        d1 += time.perf_counter() - t0
        v1 += 1
    return {"value": views / dt, "unit": "receiver-views/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{reps} x the first {n} of {wl.rx.shape[0]} receivers, full grid, {mode} mode, FP64 C "
                      f"oracle, {dt:.1f} s wall",
            "one_thread": {"value": v1 / d1, "unit": "receiver-views/s", "cores": 1,
                           "sample": f"{v1} x the first receiver, {d1:.1f} s wall"}}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the receiver-sharded "
              "multi-GPU layout is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
    wl, res = gpu_part(args)
    head = res[args.mode]
    workload = f"{args.config} {args.mode.upper()}"
    out = {
        "metric": METRIC,
        "value": head["rx_views_per_s"],
        "unit": "receiver-views/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "dtype_note": "FP32 inputs, outputs, projection keys and compositing (FP64 projection terms); the pair "
                      "MLP's layer 2 and fused layer-1 Gaussian term as split FP16 (hi + lo, three FP16 MFMA "
                      "products, ~2^-21 relative per product) with FP32 accumulation; fused.mlp_fp32 times the "
                      "FP32-MFMA variant (RXGS_MLP_FP32=1)",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {wl.scene.K} Gaussians, {wl.rx.shape[0]} receivers, "
                               f"{wl.grid.H}x{wl.grid.W} grid, MLP radiance, {args.mode.upper()}-mode views",
                   "gaussians": wl.scene.K, "receivers": int(wl.rx.shape[0]), "grid": [wl.grid.H, wl.grid.W],
                   "mode": args.mode},
        "fused": head,
        "other_modes": {k: v for k, v in res.items() if k != args.mode},
        "roofline": roofline_for(head, args.mode, workload, wl.scene.K),
        "stage_roofline": stage_rooflines(head, args.mode, wl.scene.K),
    }
    if not args.no_train:
        out["train_step"] = train_step_part(args)
    if not args.no_scale:
        out["scale"] = scale_part(args)
    if not args.no_rxcond:
        out["rxcond"] = rxcond_part(args)
    if not args.no_serve:
        out["serving"] = serving_part(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, wl, args.mode)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
