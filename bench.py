#!/usr/bin/env python3
"""Benchmark of the gfx950 projective pointmap matcher (MASt3R-SLAM, Sec. 3.2).

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step matches one 512x384 pair (196,608 query pixels, D = 24 descriptors,
10 LM iterations, refine radius 3, confidences gated at 1.5) with
m3s_match_fwd: ray-image prep plus the fused LM / refine / gate kernel.  Steps
cycle through a pool of 8 distinct pairs (~380 MB of inputs, more than the
256 MB Infinity Cache) so that inputs stream from HBM.  `value` is forward
pixel matches per second over K timed steps (inputs resident in HBM).

Further legs, reported in the same JSON line:
  fwd_bwd        forward (with xhat) then the implicit-adjoint backward per pair;
  fwd_bwd_batched the differentiation workload: 16 edges at 512x384, one batched
                 forward then one batched backward per step, against the per-pair loop;
  tracking_c2f   tracking-mode matching: previous-frame initial pixels and the
                 coarse-to-fine refine over 2 and 3 levels;
  batched        64 edges at 512x384 in one persistent hipGraph launch
                 (autotuned) vs a loop of per-pair launches on the same GPU;
  batched_uneven 96 edges of mixed resolution (512x384, 384x512, 512x288),
                 K in 5..15 and r in 2..4 per edge, same comparison;
  roofline       the forward kernel's algorithmic bytes over its average
                 duration, timed live with hipEvents around each launch;
  roofline_alu   the same launch's wave64 VALU instructions (counted by
                 rocprofv3, committed profile) over that duration, against
                 the issue rate of 256 CUs x 4 SIMDs at 2.4 GHz;
  track_fuse     the tracking pose solve (10 Gauss-Newton iterations) and the
                 canonical pointmap fusion of one 512x384 keyframe (Sec. 3.3);
  backend        Gauss-Newton over 32 keyframe poses at 512x384 with 65 edges
                 (Sec. 3.5), 10 iterations;
  cpu_baseline   the FP64 oracle on the host cores, on a bounded sample.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "pixel matches/sec (512x384 pair, 10 LM iters, r=3 refine); fwd+bwd matches/sec"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per query of the forward path (D = 24, confidences on):
# X^i_i 12 + X^j_i 12 + D^i_i 96 + D^j_i 96 + Q 8 + outputs p 8, idx 4, valid 1, theta 4.
FWD_BYTES_PER_QUERY = 12 + 12 + 8 * 24 + 8 + 8 + 4 + 1 + 4
# Backward per query: grad_p 8 + grad_xhat 12 + p 8 + valid 1 + X^j_i 12 + X^i_i 12
# + dX^j_i 12 + dX^i_i 12 + its zero fill 12; forward with xhat adds 12.
BWD_BYTES_PER_QUERY = 8 + 12 + 8 + 1 + 12 + 12 + 12 + 12 + 12
# Pose-solve accumulation per match: moving point 12 + measured point 12 + idx 4
# + valid 1 + two confidences 8.
POSE_BYTES_PER_MATCH = 12 + 12 + 4 + 1 + 4 + 4
# Fusion per pixel: read canonical point 12, confidence 4, frame point 12,
# confidence 4; write point 12, confidence 4.
FUSE_BYTES_PER_PIXEL = 12 + 4 + 12 + 4 + 12 + 4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


COUNTERS_FILE = os.path.join(ROOT, "profiles", "fwd_kernels_512x384_hbm_counters.md")
VALU_FILE = os.path.join(ROOT, "profiles", "fwd_kernels_512x384_valu_l2.md")
# wave64 VALU instructions issued per second at most: 256 CUs x 4 SIMDs x 2.4 GHz,
# one instruction per SIMD every 4 cycles (16 lanes per cycle).
VALU_PEAK_GINST = 256 * 4 * 2.4 / 4


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("m3s_kernels.hip", "m3s_device.h"):
        with open(os.path.join(ROOT, "paper_2412_12392_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_valu_per_wave(kernel: str):
    """VALU instructions per wave of `kernel` from the committed rocprofv3
    counter summary (SQ_INSTS_VALU / SQ_WAVES), or None when the summary is
    missing or was taken from different kernel sources."""
    try:
        text = open(VALU_FILE).read()
    except OSError:
        return None
    src = [l.split(":", 1)[1].strip() for l in text.splitlines() if l.startswith("source_sha256_16:")]
    if not src or src[0] != kernel_source_hash():
        return None
    for l in text.splitlines():
        cells = [c.strip() for c in l.strip().strip("|").split("|")]
        if len(cells) >= 3 and cells[0] == kernel:
            return float(cells[2])
    return None


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), or None when
    the summary is missing or was taken from different kernel sources."""
    try:
        text = open(COUNTERS_FILE).read()
    except OSError:
        return None
    src = [l.split(":", 1)[1].strip() for l in text.splitlines() if l.startswith("source_sha256_16:")]
    if not src or src[0] != kernel_source_hash():
        return None
    for l in text.splitlines():
        if l.startswith("traffic_bytes ") and l.split("=")[0].split(" ", 1)[1].strip() == kernel:
            return int(l.split("=")[1])
    return None


class PreparedPair:
    """Device tensors and pre-built ctypes argument blocks of one pair."""

    def __init__(self, m3s, lib, pair, device, want_xhat=False, K=None, r=None):
        import torch
        from paper_2412_12392_amd import _lib, binding as M
        t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(device)
        self.H, self.W = pair.H, pair.W
        self.t = dict(Xii=t(pair.Xii), Xji=t(pair.Xji), Dii=t(pair.Dii), Dji=t(pair.Dji), Qii=t(pair.Qii),
                      Qji=t(pair.Qji))
        self.res = M._alloc_outputs(pair.H, pair.W, device, True, want_xhat)
        self.pair_c = M._pair(self.t["Xii"], self.t["Xji"], self.t["Dii"], self.t["Dji"],
                                          self.t["Qii"], self.t["Qji"], None)
        self.out_c = M._outputs(self.res)
        self.prm = _lib.default_params(lib, max_iter=K if K is not None else pair.K,
                                       refine_radius=r if r is not None else pair.r)
        self.K, self.r = self.prm.max_iter, self.prm.refine_radius


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--pool", type=int, default=8, help="distinct 512x384 pairs cycled through")
    ap.add_argument("--only-main", action="store_true", help="time only the single-pair forward leg")
    ap.add_argument("--legs", default="fwd_bwd,tracking_c2f,batched,track_fuse,backend",
                    help="comma-separated further legs to run after the single-pair forward")
    ap.add_argument("--skip-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--phases-only", action="store_true",
                    help="run only the per-phase leg: the forward at (K, r) in (0,0), (10,0), (0,3), (10,3), "
                         "single pair and 64-edge batch, four launches each in that order")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (for HBM counter scaling)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the edges of a keyframe graph "
              "would shard across GPUs with no exchange in the forward); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2412_12392_amd as m3s
    from paper_2412_12392_amd import _lib
    lib = m3s.load_library()
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    props = torch.cuda.get_device_properties(dev)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream

    if args.phases_only:
        print(json.dumps({"phases": phases_leg(m3s, lib, _lib, dev, sp)}), flush=True)
        return

    # ------------------------------------------------------------ single pair
    t0 = time.time()
    pool_pairs = [synth.make_pair(384, 512, 2000 + k, K=10, r=3, conf=True) for k in range(args.pool)]
    log("generated %d pairs in %.1fs" % (len(pool_pairs), time.time() - t0))
    pool = [PreparedPair(m3s, lib, p, dev) for p in pool_pairs]
    N = pool[0].H * pool[0].W
    ws = torch.empty(lib.m3s_workspace_bytes(ctypes.byref(pool[0].pair_c), ctypes.byref(pool[0].prm)),
                     dtype=torch.uint8, device=dev)
    wsp, wsn = ws.data_ptr(), ws.numel()

    def fwd_step(k):
        P = pool[k % len(pool)]
        st = lib.m3s_match_fwd(ctypes.byref(P.pair_c), ctypes.byref(P.prm), ctypes.byref(P.out_c), wsp, wsn, sp)
        if st:
            _lib.check(lib, "m3s_match_fwd", st)

    for k in range(args.warmup):
        fwd_step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        fwd_step(k)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    value = N * args.steps / el
    ms_per_step = el / args.steps * 1e3
    log("fwd: %.3f ms/step, %.3e matches/s" % (ms_per_step, value))

    # Same steps with hipEvents around each kernel: the forward kernel's own duration.
    lib.m3s_timing_reset()
    lib.m3s_timing_enable(1)
    for k in range(args.steps):
        fwd_step(k)
    torch.cuda.synchronize()
    lib.m3s_timing_enable(0)
    kt = {}
    for name in ("prep", "fwd"):
        tot, cnt = ctypes.c_double(), ctypes.c_int64()
        _lib.check(lib, "m3s_timing_read", lib.m3s_timing_read(name.encode(), ctypes.byref(tot), ctypes.byref(cnt)))
        kt[name] = tot.value / max(cnt.value, 1)
    alg_bytes = FWD_BYTES_PER_QUERY * N
    achieved = alg_bytes / (kt["fwd"] * 1e-3) / 1e9
    traffic_bytes = measured_traffic("fwd_f16_kernel<16, 16, false>")
    traffic = None if traffic_bytes is None else round(traffic_bytes / (kt["fwd"] * 1e-3) / 1e9, 1)
    roofline = {"bound": "hbm", "kernel": "fwd_f16_kernel<16,16>", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "traffic_bytes_per_launch": traffic_bytes,
                "algorithmic_bytes_per_launch": alg_bytes,
                "kernel_avg_us": round(kt["fwd"] * 1e3, 2), "prep_avg_us": round(kt["prep"] * 1e3, 2),
                "path_achieved_GBs": round(alg_bytes / ((kt["fwd"] + kt["prep"]) * 1e-3) / 1e9, 1)}
    log("kernel timing: fwd %.2f us, prep %.2f us" % (kt["fwd"] * 1e3, kt["prep"] * 1e3))

    # Forward kernel time per tile configuration (0-2: refine from global
    # memory; 3-4: refine region staged in LDS; 5: fp16 pre-filter; 6: the same
    # with 8x8 one-wave tiles), same pool and steps.
    sweep = {}
    for tc, remap in [(t, "1") for t in range(7)] + [(3, "0"), (5, "0"), (6, "0")]:
        m3s.set_launch(tile_config=tc, xcd_remap=int(remap))
        lib.m3s_timing_reset()
        lib.m3s_timing_enable(1)
        for k in range(min(args.steps, 30)):
            fwd_step(k)
        torch.cuda.synchronize()
        lib.m3s_timing_enable(0)
        tot, cnt = ctypes.c_double(), ctypes.c_int64()
        lib.m3s_timing_read(b"fwd", ctypes.byref(tot), ctypes.byref(cnt))
        sweep["%d%s" % (tc, "" if remap == "1" else "_no_xcd_remap")] = round(tot.value / max(cnt.value, 1) * 1e3, 2)
    m3s.set_launch()
    roofline["fwd_us_by_tile_config"] = sweep
    log("fwd kernel us by tile config:", sweep)

    out = {"metric": METRIC, "value": round(value, 1), "unit": "matches/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "single pair 512x384 (W x H), D=24, K=10 LM iterations, r=3 refine, "
                                  "confidences gated at 1.5, identity init",
                      "queries_per_step": N, "pool_pairs": len(pool), "device": props.name,
                      "gcn_arch": getattr(props, "gcnArchName", "")},
           "roofline": roofline,
           # The paper's own timings on its own hardware (matching table, Sec. 4): context, not a target.
           "paper_context": {"hardware": "NVIDIA RTX 4090", "match_ms_projection": 0.5,
                             "match_ms_projection_refine": 2.0, "system_fps": 15,
                             "this_ms_per_step": round(ms_per_step, 5)}}
    vpw = measured_valu_per_wave("fwd_f16_kernel<16, 16, false>")
    if vpw is not None:
        waves = ((pool[0].W + 15) // 16) * ((pool[0].H + 15) // 16) * 4
        ach = vpw * waves / (kt["fwd"] * 1e-3) / 1e9
        out["roofline_alu"] = {"bound": "alu", "kernel": "fwd_f16_kernel<16,16>", "achieved": round(ach, 1),
                               "peak": VALU_PEAK_GINST, "unit": "G wave64 VALU instructions/s",
                               "frac": round(ach / VALU_PEAK_GINST, 4), "valu_instructions_per_wave": vpw,
                               "waves_per_launch": waves}

    if not args.only_main:
        legs = set(args.legs.split(","))
        if "fwd_bwd" in legs:
            out["fwd_bwd"] = fwd_bwd_leg(m3s, lib, _lib, pool_pairs, dev, sp, args)
            out["fwd_bwd_batched"] = fwd_bwd_batched_leg(m3s, lib, _lib, dev, args)
        if "tracking_c2f" in legs:
            out["tracking_c2f"] = tracking_c2f_leg(m3s, lib, _lib, pool_pairs, dev, sp, args)
        if "batched" in legs:
            out["batched"] = batched_leg(m3s, lib, _lib, synth.batched_uniform, dev, args,
                                         "64 edges 512x384, K=10, r=3")
            out["batched_uneven"] = batched_leg(m3s, lib, _lib, synth.batched_uneven, dev, args,
                                                "96 edges: 40x 512x384, 32x 384x512, 24x 512x288; K 5..15, r 2..4")
        if "track_fuse" in legs:
            out["track_fuse"] = track_fuse_leg(m3s, lib, dev, args)
        if "backend" in legs:
            out["backend"] = backend_leg(m3s, lib, dev, args)
    if args.copy_calibration:
        out["copy_calibration"] = copy_calibration(torch, dev)
    if not args.skip_cpu:
        # Pair 0 once more in the default launch (the legs above changed tile
        # configurations), for the agreement statement on the oracle's output.
        fwd_step(0)
        torch.cuda.synchronize()
        out["cpu_baseline"], ora = cpu_baseline(pool_pairs[0], args.cpu_seconds)
        out["parity"] = parity_statement(pool[0].res, ora)
        log("parity vs oracle:", out["parity"])
    print(json.dumps(out), flush=True)


PHASE_VARIANTS = [(0, 0), (10, 0), (0, 3), (10, 3)]


def phases_leg(m3s, lib, _lib, dev, sp, pairs=None):
    """The forward at LM iterations K and refine radius r of PHASE_VARIANTS, so
    that per-phase costs follow by difference (K=0, r=0: setup, initial sample,
    staging and gates; the K and r increments: the LM iterations and the
    window refine).  For each variant, in this order: one 512x384 pair
    (m3s_match_fwd, default launch) 1 + 3 launches, then the 64-edge batch
    (m3s_match_batched, eager, default tile configuration) 1 + 3 launches,
    each timed with hipEvents.  Instruction counters of the same launches come
    from rocprofv3 (dispatch order)."""
    import torch
    pairs = pairs if pairs is not None else synth.batched_uniform()
    edges = []
    for p in pairs:
        t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        edges.append(m3s.EdgeInput(t(p.Xii), t(p.Xji), t(p.Dii), t(p.Dji), t(p.Qii), t(p.Qji), None, -1, -1))
    table, outs = m3s.make_edges(edges)
    n = len(edges)
    queries = sum(p.H * p.W for p in pairs)
    out = []
    for K, r in PHASE_VARIANTS:
        prm = _lib.default_params(lib, max_iter=K, refine_radius=r)
        nb = lib.m3s_batched_workspace_bytes(table, n, ctypes.byref(prm))
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        pw = torch.empty(lib.m3s_workspace_bytes(ctypes.byref(table[0].in_), ctypes.byref(prm)), dtype=torch.uint8,
                         device=dev)

        def single():
            st = lib.m3s_match_fwd(ctypes.byref(table[0].in_), ctypes.byref(prm), ctypes.byref(table[0].out),
                                   pw.data_ptr(), pw.numel(), sp)
            _lib.check(lib, "m3s_match_fwd", st)

        def batch():
            st = lib.m3s_match_batched(table, n, ctypes.byref(prm), 0, ws.data_ptr(), ws.numel(), sp)
            _lib.check(lib, "m3s_match_batched", st)

        rec = {"K": K, "r": r}
        for name, fn, timer in (("single_fwd_us", single, "fwd"), ("batched_fwd_us", batch, "batched_fwd")):
            fn()
            torch.cuda.synchronize()
            lib.m3s_timing_reset()
            lib.m3s_timing_enable(1)
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            lib.m3s_timing_enable(0)
            ms, _ = _timer(lib, timer)
            rec[name] = round(ms * 1e3, 2)
        rec["batched_matches_per_s"] = round(queries / (rec["batched_fwd_us"] * 1e-6), 1)
        log("phases:", rec)
        out.append(rec)
        del ws, pw
    return {"workload": "64 edges 512x384 (batched) and edge 0 alone (single pair); D=24, confidences",
            "queries_batched": queries, "variants": out}


def tracking_c2f_leg(m3s, lib, _lib, pool_pairs, dev, sp, args):
    """Tracking-mode matching (Sec. 3.2): each 512x384 pair of the pool starts
    from the previous frame's matches, stood in for by the generator's true
    projection plus N(0, 1.5^2) px noise, and refines coarse to fine over L = 2
    and L = 3 levels (r = 3, K = 10).  Single-pair forward per step, kernel
    time from hipEvents; algorithmic bytes per query 241 + 8 (p_init)."""
    import torch
    rng = np.random.Generator(np.random.PCG64(77))
    pinit = [torch.from_numpy((p.proj + rng.normal(0, 1.5, size=p.proj.shape)).astype(np.float32)).to(dev)
             for p in pool_pairs]
    pool = [PreparedPair(m3s, lib, p, dev) for p in pool_pairs]
    for P, pi in zip(pool, pinit):
        P.pair_c.p_init = pi.data_ptr()
    N = pool[0].H * pool[0].W
    ws = torch.empty(lib.m3s_workspace_bytes(ctypes.byref(pool[0].pair_c), ctypes.byref(pool[0].prm)),
                     dtype=torch.uint8, device=dev)
    out = {"workload": "512x384 pairs, p_init = previous-frame matches (projection + N(0, 1.5^2) px), K=10, r=3, "
                       "coarse-to-fine refine", "bytes_per_query": FWD_BYTES_PER_QUERY + 8}
    for L in (2, 3):
        prm = _lib.default_params(lib, refine_levels=L)

        def step(k):
            P = pool[k % len(pool)]
            st = lib.m3s_match_fwd(ctypes.byref(P.pair_c), ctypes.byref(prm), ctypes.byref(P.out_c), ws.data_ptr(),
                                   ws.numel(), sp)
            _lib.check(lib, "m3s_match_fwd", st)

        for k in range(5):
            step(k)
        torch.cuda.synchronize()
        m3s.path_counters(reset=True)
        steps = max(10, args.steps // 2)
        t0 = time.perf_counter()
        for k in range(steps):
            step(k)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        counts = m3s.path_counters(reset=True)
        lib.m3s_timing_reset()
        lib.m3s_timing_enable(1)
        for k in range(steps):
            step(k)
        torch.cuda.synchronize()
        lib.m3s_timing_enable(0)
        fwd_ms, _ = _timer(lib, "fwd")
        alg = (FWD_BYTES_PER_QUERY + 8) * N
        out["L%d" % L] = {"matches_per_s": round(N / el, 1), "ms_per_step": round(el * 1e3, 5),
                          "fwd_kernel_us": round(fwd_ms * 1e3, 2),
                          "fwd_algorithmic_GBs": round(alg / (fwd_ms * 1e-3) / 1e9, 1),
                          "fwd_frac_of_hbm_peak": round(alg / (fwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "global_scan_tile_levels_per_step": round(counts["refine_global"] / steps, 1),
                          "banded_tile_levels_per_step": round(counts["refine_bands"] / steps, 1)}
    log("tracking_c2f:", out)
    return out


def fwd_bwd_leg(m3s, lib, _lib, pool_pairs, dev, sp, args):
    import torch
    pool = [PreparedPair(m3s, lib, p, dev, want_xhat=True) for p in pool_pairs]
    N = pool[0].H * pool[0].W
    ws = torch.empty(lib.m3s_workspace_bytes(ctypes.byref(pool[0].pair_c), ctypes.byref(pool[0].prm)),
                     dtype=torch.uint8, device=dev)
    g = torch.Generator(device="cpu").manual_seed(0)
    grad_p = torch.randn((pool[0].H, pool[0].W, 2), generator=g).to(dev)
    grad_x = torch.randn((pool[0].H, pool[0].W, 3), generator=g).to(dev)
    gXi = torch.empty((pool[0].H, pool[0].W, 3), device=dev)
    gXj = torch.empty_like(gXi)
    bwd_pairs = [_lib.Pair(P.H, P.W, 0, P.t["Xii"].data_ptr(), P.t["Xji"].data_ptr(), 0, 0, 0, 0, 0) for P in pool]

    def step(k):
        P = pool[k % len(pool)]
        st = lib.m3s_match_fwd(ctypes.byref(P.pair_c), ctypes.byref(P.prm), ctypes.byref(P.out_c), ws.data_ptr(),
                               ws.numel(), sp)
        _lib.check(lib, "m3s_match_fwd", st)
        st = lib.m3s_match_bwd(ctypes.byref(bwd_pairs[k % len(pool)]), ctypes.byref(P.out_c), grad_p.data_ptr(),
                               grad_x.data_ptr(), gXi.data_ptr(), gXj.data_ptr(), sp)
        _lib.check(lib, "m3s_match_bwd", st)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    lib.m3s_timing_reset()
    lib.m3s_timing_enable(1)
    for k in range(min(args.steps, 20)):
        step(k)
    torch.cuda.synchronize()
    lib.m3s_timing_enable(0)
    kt = {}
    for name in ("prep", "fwd", "fill", "bwd"):
        tot, cnt = ctypes.c_double(), ctypes.c_int64()
        lib.m3s_timing_read(name.encode(), ctypes.byref(tot), ctypes.byref(cnt))
        kt[name + "_avg_us"] = round(tot.value / max(cnt.value, 1) * 1e3, 2)
    bwd_us = kt["bwd_avg_us"] + kt["fill_avg_us"]
    res = {"workload": "512x384 pair: forward with xhat, then backward (grad_p, grad_xhat)",
           "matches_per_s": round(N * args.steps / el, 1), "ms_per_step": round(el / args.steps * 1e3, 5),
           "kernels": kt,
           "bwd_achieved_GBs": round(BWD_BYTES_PER_QUERY * N / (bwd_us * 1e-6) / 1e9, 1)}
    # Whole step: forward (with xhat) plus backward bytes over the measured step time.
    step_gbs = (FWD_BYTES_PER_QUERY + 12 + BWD_BYTES_PER_QUERY) * N * args.steps / el / 1e9
    res["step_algorithmic_GBs"] = round(step_gbs, 1)
    res["step_frac_of_hbm_peak"] = round(step_gbs / HBM_PEAK_GBS, 4)
    log("fwd+bwd:", res)
    return res


def fwd_bwd_batched_leg(m3s, lib, _lib, dev, args):
    """The differentiation workload: 16 edges at 512x384 per step, one batched
    forward (with xhat; one persistent launch) then one batched backward
    (zero-fill + static-band launch) to dL/dX^i_i and dL/dX^j_i for L = sum
    over valid matches of |xhat - x|^2 (grad_xhat = 2 (xhat - x) on valid
    queries, from one forward before timing).  Both calls are timed with the
    library's hipGraphs (M3S_BATCH_GRAPH) and with eager launches; the step
    figure is the faster of the two."""
    import torch
    t0 = time.time()
    pairs = [synth.config_pair(5, e) for e in range(16)]
    log("fwd_bwd_batched leg: %d edges generated in %.1fs" % (len(pairs), time.time() - t0))
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    edges = [m3s.EdgeInput(t(p.Xii), t(p.Xji), t(p.Dii), t(p.Dji), t(p.Qii), t(p.Qji), None, p.K, p.r) for p in pairs]
    queries = sum(p.H * p.W for p in pairs)
    n = len(edges)
    prm = m3s.params()
    table, outs = m3s.make_edges(edges, want_xhat=True)
    ws = torch.empty(lib.m3s_batched_workspace_bytes(table, n, ctypes.byref(prm)), dtype=torch.uint8, device=dev)
    s = torch.cuda.Stream()
    fflags = _lib.M3S_BATCH_GRAPH | _lib.M3S_BATCH_AUTOTUNE

    gflag = [_lib.M3S_BATCH_GRAPH]  # submission mode of fwd() and bwd(): GRAPH or 0 (eager)

    def fwd():
        fl = _lib.M3S_BATCH_AUTOTUNE | gflag[0]
        st = lib.m3s_match_batched(table, n, ctypes.byref(prm), fl, ws.data_ptr(), ws.numel(), s.cuda_stream)
        _lib.check(lib, "m3s_match_batched", st)

    with torch.cuda.stream(s):
        fwd()
    s.synchronize()
    bins = []
    for e, o in zip(edges, outs):
        gx = (2.0 * (o.xhat - e.Xji) * o.valid[..., None].float()).contiguous()
        bins.append(m3s.BwdEdgeInput(e.Xii, e.Xji, o.p, o.valid, torch.zeros_like(o.p), gx))
    btable, grads = m3s.make_bwd_edges(bins)
    wsb = torch.empty(lib.m3s_bwd_batched_workspace_bytes(n), dtype=torch.uint8, device=dev)

    def bwd():
        st = lib.m3s_match_bwd_batched(btable, n, gflag[0], wsb.data_ptr(), wsb.numel(), s.cuda_stream)
        _lib.check(lib, "m3s_match_bwd_batched", st)

    def step():
        fwd()
        bwd()

    steps = max(5, args.steps // 5)
    mode_ms = {}
    for mode, gf in (("graph", _lib.M3S_BATCH_GRAPH), ("eager", 0)):
        gflag[0] = gf
        with torch.cuda.stream(s):
            for _ in range(3):
                step()
        s.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(s):
            for _ in range(steps):
                step()
        s.synchronize()
        mode_ms[mode] = (time.perf_counter() - t0) / steps * 1e3
    best_mode = min(mode_ms, key=mode_ms.get)
    el = mode_ms[best_mode] / 1e3
    gflag[0] = _lib.M3S_BATCH_GRAPH
    lib.m3s_timing_reset()
    lib.m3s_timing_enable(1)
    with torch.cuda.stream(s):
        for _ in range(3):
            step()
    s.synchronize()
    lib.m3s_timing_enable(0)
    fg, _ = _timer(lib, "batched_graph")
    bg, _ = _timer(lib, "batched_bwd_graph")
    # Per-pair loop of the same work on the same stream, for comparison.
    pw = torch.empty(lib.m3s_workspace_bytes(ctypes.byref(table[0].in_), ctypes.byref(prm)), dtype=torch.uint8,
                     device=dev)
    bpairs = [_lib.Pair(e.Xii.shape[0], e.Xii.shape[1], 0, e.Xii.data_ptr(), e.Xji.data_ptr(), 0, 0, 0, 0, 0)
              for e in edges]

    def loop():
        for k in range(n):
            st = lib.m3s_match_fwd(ctypes.byref(table[k].in_), ctypes.byref(prm), ctypes.byref(table[k].out),
                                   pw.data_ptr(), pw.numel(), s.cuda_stream)
            _lib.check(lib, "m3s_match_fwd", st)
            st = lib.m3s_match_bwd(ctypes.byref(bpairs[k]), ctypes.byref(table[k].out), bins[k].grad_p.data_ptr(),
                                   bins[k].grad_xhat.data_ptr(), grads[k][0].data_ptr(), grads[k][1].data_ptr(),
                                   s.cuda_stream)
            _lib.check(lib, "m3s_match_bwd", st)

    with torch.cuda.stream(s):
        loop()
    s.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(s):
        for _ in range(max(3, steps // 2)):
            loop()
    s.synchronize()
    el_p = (time.perf_counter() - t0) / max(3, steps // 2)
    step_bytes = (FWD_BYTES_PER_QUERY + 12 + BWD_BYTES_PER_QUERY) * queries
    res = {"workload": "16 edges 512x384 (W x H), K=10, r=3, confidences: batched forward with xhat then batched "
                       "implicit-adjoint backward, L = sum of squared matched-point distances",
           "edges": n, "queries": queries, "matches_per_s": round(queries / el, 1), "ms_per_step": round(el * 1e3, 4),
           "submission": best_mode, "ms_by_submission": {k: round(v, 4) for k, v in mode_ms.items()},
           "fwd_graph_ms_events": round(fg, 4), "bwd_graph_ms_events": round(bg, 4),
           "per_pair_loop_matches_per_s": round(queries / el_p, 1), "per_pair_loop_ms": round(el_p * 1e3, 4),
           "speedup_vs_per_pair": round(el_p / el, 3),
           "step_algorithmic_GBs": round(step_bytes / el / 1e9, 1),
           "step_frac_of_hbm_peak": round(step_bytes / el / 1e9 / HBM_PEAK_GBS, 4),
           "bwd_algorithmic_GBs": round(BWD_BYTES_PER_QUERY * queries / (bg * 1e-3) / 1e9, 1),
           "bwd_frac_of_hbm_peak": round(BWD_BYTES_PER_QUERY * queries / (bg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    log("fwd_bwd_batched:", res)
    del ws, wsb, pw, outs, edges, grads
    torch.cuda.empty_cache()
    return res


def batched_leg(m3s, lib, _lib, make_pairs, dev, args, label):
    import torch
    t0 = time.time()
    pairs = make_pairs()
    log("batched leg %s: %d edges generated in %.1fs" % (label, len(pairs), time.time() - t0))
    edges = []
    for p in pairs:
        t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        edges.append(m3s.EdgeInput(t(p.Xii), t(p.Xji), t(p.Dii), t(p.Dji), t(p.Qii), t(p.Qji), None, p.K, p.r))
    queries = sum(p.H * p.W for p in pairs)
    prm = m3s.params()
    table, outs = m3s.make_edges(edges)
    n = len(edges)
    nbytes = lib.m3s_batched_workspace_bytes(table, n, ctypes.byref(prm))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    s = torch.cuda.Stream()
    flags = _lib.M3S_BATCH_GRAPH | _lib.M3S_BATCH_AUTOTUNE

    def call(fl=flags):
        st = lib.m3s_match_batched(table, n, ctypes.byref(prm), fl, ws.data_ptr(), ws.numel(), s.cuda_stream)
        _lib.check(lib, "m3s_match_batched", st)

    steps = max(3, args.steps // 10)
    with torch.cuda.stream(s):
        for _ in range(max(2, args.warmup // 5)):
            call()
    s.synchronize()
    launch = m3s.last_batched_launch()
    # Both submission modes, same tuned launch: the library's hipGraph
    # (M3S_BATCH_GRAPH) and eager launches; the step figure is the faster.
    mode_ms = {}
    for mode, fl in (("graph", flags), ("eager", _lib.M3S_BATCH_AUTOTUNE)):
        with torch.cuda.stream(s):
            call(fl)
        s.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(s):
            for _ in range(steps):
                call(fl)
        s.synchronize()
        mode_ms[mode] = (time.perf_counter() - t0) / steps * 1e3
    best_mode = min(mode_ms, key=mode_ms.get)
    el_b = mode_ms[best_mode] / 1e3
    lib.m3s_timing_reset()
    lib.m3s_timing_enable(1)
    with torch.cuda.stream(s):
        call()
    s.synchronize()
    lib.m3s_timing_enable(0)
    tot, cnt = ctypes.c_double(), ctypes.c_int64()
    lib.m3s_timing_read(b"batched_graph", ctypes.byref(tot), ctypes.byref(cnt))
    graph_ms = tot.value / max(cnt.value, 1)

    # Per-pair loop over the same edges on the same stream.
    pw = torch.empty(max(lib.m3s_workspace_bytes(ctypes.byref(table[k].in_), ctypes.byref(prm)) for k in range(n)),
                     dtype=torch.uint8, device=dev)
    prms = [_lib.default_params(lib, max_iter=e.max_iter, refine_radius=e.refine_radius) for e in edges]

    def loop():
        for k in range(n):
            st = lib.m3s_match_fwd(ctypes.byref(table[k].in_), ctypes.byref(prms[k]), ctypes.byref(table[k].out),
                                   pw.data_ptr(), pw.numel(), s.cuda_stream)
            _lib.check(lib, "m3s_match_fwd", st)

    with torch.cuda.stream(s):
        loop()
    s.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(s):
        for _ in range(steps):
            loop()
    s.synchronize()
    el_p = (time.perf_counter() - t0) / steps
    res = {"workload": label, "edges": n, "queries": queries,
           "batched_matches_per_s": round(queries / el_b, 1), "batched_ms": round(el_b * 1e3, 4),
           "submission": best_mode, "ms_by_submission": {k: round(v, 4) for k, v in mode_ms.items()},
           "graph_launch_ms_events": round(graph_ms, 4),
           "per_pair_loop_matches_per_s": round(queries / el_p, 1), "per_pair_loop_ms": round(el_p * 1e3, 4),
           "speedup_vs_per_pair": round(el_p / el_b, 3), "launch": launch,
           "algorithmic_GBs": round(queries * FWD_BYTES_PER_QUERY / el_b / 1e9, 1),
           "frac_of_hbm_peak": round(queries * FWD_BYTES_PER_QUERY / el_b / 1e9 / HBM_PEAK_GBS, 4)}
    log("batched:", res)
    del ws, pw, outs, edges
    torch.cuda.empty_cache()
    return res


def _timer(lib, name):
    tot, cnt = ctypes.c_double(), ctypes.c_int64()
    lib.m3s_timing_read(name.encode(), ctypes.byref(tot), ctypes.byref(cnt))
    return tot.value / max(cnt.value, 1), cnt.value


def track_fuse_leg(m3s, lib, dev, args):
    """Tracking pose solve + fusion of one 512x384 keyframe (Sec. 3.3)."""
    import torch
    H, W = 384, 512
    tp = synth.make_tracking(H, W, 5000, noise=1e-3, outlier_frac=0.05)
    fp = synth.make_fusion(H, W, 5001)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    prob = (t(tp.Xk), t(tp.Xf), t(tp.idx.astype(np.int32)), t(tp.valid.astype(np.uint8)), t(tp.Qf), t(tp.Qk))
    Xc, Cc, X, C = t(fp.Xc), t(fp.Cc), t(fp.X), t(fp.C)
    I34 = torch.tensor(np.concatenate([np.eye(3), np.zeros((3, 1))], 1), dtype=torch.float32, device=dev)
    T = I34.clone()
    prm = m3s.track_params()

    def step():
        T.copy_(I34)
        m3s.track_pose(*prob, T, prm)
        m3s.fuse_pointmap(Xc, Cc, X, C, T)

    steps = max(5, args.steps // 5)
    for _ in range(3):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    lib.m3s_timing_reset()
    lib.m3s_timing_enable(1)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    lib.m3s_timing_enable(0)
    # The same frame captured once into a graph and replayed.
    g = torch.cuda.CUDAGraph()
    gs = torch.cuda.Stream()
    gs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(gs):
        step()
    torch.cuda.current_stream().wait_stream(gs)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        step()
    for _ in range(3):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    el_graph = (time.perf_counter() - t0) / steps
    ac_ms, _ = _timer(lib, "track_step")
    so_ms, _ = _timer(lib, "track_final")
    fu_ms, _ = _timer(lib, "fuse")
    n_match = int(tp.valid.sum())
    iters = prm.iters + 1
    out = {"workload": "512x384 keyframe: tracking pose solve (10 Gauss-Newton iterations + final cost) then "
                       "pointmap fusion; noise 1e-3, 5% outliers",
           "ms_per_frame": round(el * 1e3, 4), "ms_per_frame_graph": round(el_graph * 1e3, 4),
           "track_step_avg_us": round(ac_ms * 1e3, 2), "track_final_avg_us": round(so_ms * 1e3, 2),
           "step_launches_per_frame": iters,
           "match_evaluations_per_s": round(n_match * iters / el, 1),
           "track_step_algorithmic_GBs": round(POSE_BYTES_PER_MATCH * H * W / (ac_ms * 1e-3) / 1e9, 1),
           "fuse_avg_us": round(fu_ms * 1e3, 2),
           "fuse_algorithmic_GBs": round(FUSE_BYTES_PER_PIXEL * H * W / (fu_ms * 1e-3) / 1e9, 1),
           "fuse_frac_of_hbm_peak": round(FUSE_BYTES_PER_PIXEL * H * W / (fu_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    log("track_fuse:", out)
    return out


def backend_leg(m3s, lib, dev, args):
    """Backend Gauss-Newton over 32 keyframes at 512x384 with 65 edges (Sec. 3.5)."""
    import torch
    N, H, W = 32, 384, 512
    t0 = time.time()
    bp = synth.make_backend(N, H, W, 6000, loops=3, scramble=False, noise=1e-3, outlier_frac=0.05)
    log("backend leg: %d keyframes, %d edges generated in %.1fs" % (N, len(bp.edges), time.time() - t0))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    prob = (t(bp.Xc), t(bp.Q), t(bp.edges), t(bp.idx), t(bp.valid.astype(np.uint8)))
    T0 = t(np.asarray(bp.T_init, np.float32))
    T = T0.clone()
    prm = m3s.backend_params()

    def step():
        T.copy_(T0)
        m3s.backend_gn(*prob, T, prm)

    steps = max(3, args.steps // 10)
    for _ in range(2):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    lib.m3s_timing_reset()
    lib.m3s_timing_enable(1)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    lib.m3s_timing_enable(0)
    g = torch.cuda.CUDAGraph()
    gs = torch.cuda.Stream()
    gs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(gs):
        step()
    torch.cuda.current_stream().wait_stream(gs)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        step()
    for _ in range(2):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    el_graph = (time.perf_counter() - t0) / steps
    acc_ms, _ = _timer(lib, "backend_accum")
    edg_ms, _ = _timer(lib, "backend_edge")
    sol_ms, _ = _timer(lib, "backend_solve")
    E = len(bp.edges)
    matches = E * H * W
    # Bytes an iteration has to read at least: every edge's idx and valid, and
    # every keyframe's points and confidences once (keyframes are shared by
    # several edges).
    alg = E * H * W * (4 + 1) + N * H * W * (12 + 4)
    out = {"workload": "%d keyframes 512x384, %d edges (neighbours both ways + loop closures), 10 Gauss-Newton "
                       "iterations, noise 1e-3, 5%% outliers" % (N, E),
           "ms_per_solve": round(el * 1e3, 4), "ms_per_solve_graph": round(el_graph * 1e3, 4),
           "match_evaluations_per_s": round(matches * (prm.iters + 1) / el, 1),
           "accum_avg_us": round(acc_ms * 1e3, 2), "edge_avg_us": round(edg_ms * 1e3, 2),
           "solve_avg_us": round(sol_ms * 1e3, 2),
           "accum_algorithmic_bytes": alg, "accum_match_bytes": POSE_BYTES_PER_MATCH * matches,
           "accum_algorithmic_GBs": round(alg / (acc_ms * 1e-3) / 1e9, 1),
           "accum_frac_of_hbm_peak": round(alg / (acc_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    log("backend:", out)
    return out


def copy_calibration(torch, dev):
    """A plain device copy of known size, for scaling HBM byte counters."""
    n = 256 << 20
    a = torch.empty(n // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"bytes_read": n, "bytes_written": n, "launches": 3}


def cpu_model() -> str:
    """The host CPU's model name (as lscpu reports it, from /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pair, seconds):
    """The FP64 oracle (OpenMP over queries) on the host cores: the median of
    5 timed runs after one warm-up, each run repeating forward passes over one
    512x384 pair for about seconds/5 of wall time, with all threads; then the
    same median with one thread (one pass per run)."""
    import oracle
    lib = oracle.load()
    N = pair.H * pair.W
    ora = oracle.match_pair(pair)  # warm-up (thread pool)

    def runs(nthreads, min_s):
        rates, calls_total, wall = [], 0, 0.0
        for _ in range(5):
            calls = 0
            t0 = time.perf_counter()
            while True:
                oracle.match_pair(pair, nthreads=nthreads)
                calls += 1
                el = time.perf_counter() - t0
                if el >= min_s:
                    break
            rates.append(N * calls / el)
            calls_total += calls
            wall += el
        return float(np.median(rates)), calls_total, wall

    all_rate, all_calls, all_wall = runs(0, seconds / 5.0)
    one_rate, one_calls, one_wall = runs(1, 0.0)
    threads = oracle.max_threads(lib)
    return {"value": round(all_rate, 1), "unit": "matches/s", "cores": threads, "kind": "oracle",
            "sample": "median of 5 runs after one warm-up, each repeating the forward over one %dx%d pair "
                      "(%d queries) for >= %.1f s: %d passes in %.1f s with %d threads; fp64 C, OpenMP over queries"
                      % (pair.W, pair.H, N, seconds / 5.0, all_calls, all_wall, threads),
            "one_thread": {"value": round(one_rate, 1), "unit": "matches/s", "cores": 1,
                           "sample": "median of 5 single passes over the same pair (%.1f s)" % one_wall},
            "host_cpus": os.cpu_count(), "cpu_model": cpu_model()}, ora


def parity_statement(res, ora):
    """This run's forward on the benchmark pair against the oracle's, on the
    matching contract: valid flags agree on >= 99.9 % of queries; p* within
    1e-3 px and theta within 1e-5 rad where both are valid; idx identical where
    both are valid, the top-two window scores differ by more than 1e-5 and p*
    is at least 1e-3 px from a rounding boundary in both axes."""
    p = res.p.cpu().numpy().astype(np.float64).reshape(-1, 2)
    idx = res.idx.cpu().numpy().astype(np.int64).reshape(-1)
    vg = res.valid.cpu().numpy().astype(bool).reshape(-1)
    th = res.theta.cpu().numpy().astype(np.float64).reshape(-1)
    po = np.asarray(ora["p"], np.float64).reshape(-1, 2)
    vo = np.asarray(ora["valid"], bool).reshape(-1)
    both = vg & vo
    frac = po - np.floor(po)
    straddle = (np.abs(frac - 0.5) < 1e-3).any(-1)
    comp = both & (np.asarray(ora["gap"]).reshape(-1) > 1e-5) & ~straddle
    agree = float((vg == vo).mean())
    dp = float(np.abs(p - po).max(-1)[both].max()) if both.any() else 0.0
    dth = float(np.abs(th - np.asarray(ora["theta"]).reshape(-1))[both].max()) if both.any() else 0.0
    mism = int((idx != np.asarray(ora["idx"]).reshape(-1))[comp].sum())
    return {"queries": int(vg.size), "valid_gpu": int(vg.sum()), "valid_oracle": int(vo.sum()),
            "valid_agreement": round(agree, 6), "max_dp_px": dp, "max_dtheta": dth,
            "idx_compared": int(comp.sum()), "idx_mismatch": mism,
            "pass": bool(agree >= 0.999 and dp <= 1e-3 and dth <= 1e-5 and mism == 0)}


if __name__ == "__main__":
    main()
