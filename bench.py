"""Benchmark of the odd-even Wilson-clover hot path on one MI355X.

A step is one pass of the path over one batch of synthetic input on the large
single-GPU lattice 48^3 x 96 (eps 0.5, c_sw 1.2, m0 -0.25, t antiperiodic):
one FP32 Schur apply y_e = D_S x_e (eq. 3) and 20 FP32 Richardson sweeps
(Alg. 4) with omega = 0.8 / |lambda_max(D_S)|.  Inputs are resident in HBM before
the timed region.  Reported:

  value          FP32 Schur-apply GB/s: algorithmic bytes of one apply (every
                 field touched once per kernel: 2208 B per even site) / apply time
  sweeps_per_s   FP32 Richardson sweeps per second
  roofline       the dominant stencil kernel's algorithmic bytes per launch / its
                 mean HIP-event duration, against 8 TB/s
  mixed_vs_fp64  time to |b - D x| / |b| <= 1e-10 on 16^3 x 32 (eps 0.5, c_sw 1.0,
                 m0 -0.2, Gaussian b) for FP64 GMRES(50) and for the same solver
                 with the operator and Richardson preconditioner in FP32; also
                 FGMRES(50) on the full D with the odd-even smoother M_nu
  multi_rhs      24^3 x 48 with 12 right-hand sides: FP32 Schur apply GB/s with the
                 autotuned register-blocked tile vs a loop of single applies
  batched        12 right-hand sides on 24^3 x 48 plus 8^4, 12^4, 16^3 x 32 with 4
                 each (eps 0.5, c_sw 1.0, m0 -0.2): all 24 systems to 1e-10 in one
                 lock-step batched solve (FP32 inner, FP64 outer) vs the same
                 systems solved one by one, mixed and plain FP64
  cpu_baseline   the FP64 NumPy oracle on the host, on a bounded sample

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-solve] [--no-batch] [--no-cpu]
       python bench.py --multi-rhs-only   (profiling run: only the 12-right-hand-side apply on 24^3 x 48,
                                           prints its own JSON, not the benchmark line)
       python bench.py --batch-only       (profiling run: that apply and the batched solves, own JSON)
       python bench.py --mrhs-only        (profiling run: only the interleaved-layout 12-right-hand-side stencil)
       python bench.py --headline-only    (profiling run: only the timed FP32 step on 48^3 x 96, own JSON)
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

METRIC = "Schur apply GB/s (% HBM peak) + smoother sweeps/s, mixed vs FP64 at 1e-10 resid"
HBM_PEAK_GBS = 8000.0
LARGE = dict(dims=(48, 48, 48, 96), eps=0.5, c_sw=1.2, m0=-0.25, seed_gauge=301, seed_vec=302)
MIXED = dict(dims=(16, 16, 16, 32), eps=0.5, c_sw=1.0, m0=-0.2, seed_gauge=201, seed_vec=202)
# (dims, right-hand sides, gauge seed); right-hand side r of a lattice uses seed + 1000 + r
BATCH = [((24, 24, 24, 48), 12, 401), ((8, 8, 8, 8), 4, 402), ((12, 12, 12, 12), 4, 403), ((16, 16, 16, 32), 4, 404)]
SWEEPS = 20
BYTES_APPLY_F32 = 2208    # per even site, FP32 links/spinors/clover, every field once per kernel
BYTES_APPLY_F64 = 4416
BYTES_APPLY_F32_L12 = 1824  # 12-real FP32 links
BYTES_APPLY_H16 = 944       # 16-bit spinors, 12-real links, clover padded to 40 slots
BYTES_APPLY_H16_C32 = 1200  # 16-bit spinors, 12-real 16-bit links, FP32 clover blocks


MODE_CODE = {"clinv": 0, "recon": 1, "apply": 2, "richardson": 3, "resid": 4, "prep": 5}
KERNEL_SOURCES = ("paper_2407_08092_amd/csrc/hop.hip", "paper_2407_08092_amd/csrc/hop_common.h",
                  "paper_2407_08092_amd/csrc/ddq_device.h",
                  "paper_2407_08092_amd/csrc/ddq_internal.h")
PROFILE = "profiles/hop_fp32_step_48x96.md"


def measured_traffic(kernel_name: str, bytes_per_launch: float):
    """Traffic past L2 per launch of a stencil kernel: its algorithmic bytes times the ratio
    of counter traffic (FETCH_SIZE x 2 + WRITE_SIZE, calibrated on a copy kernel) to
    algorithmic bytes in the committed rocprofv3 summary; None when the kernel sources
    changed since the counters were taken."""
    import hashlib

    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    cur = h.hexdigest()[:16]
    parts = kernel_name.split("_")  # hop_<mode>_<f32|f32l12|f64>[...]
    if len(parts) < 3 or parts[1] not in MODE_CODE:
        return None
    key = ("float" if parts[2].startswith("f32") else "double") + f":{MODE_CODE[parts[1]]}"
    if parts[2] == "f32l12":
        key += ":l12"
    try:
        lines = open(os.path.join(ROOT, PROFILE)).read().splitlines()
    except OSError:
        return None
    for ln in lines:
        f = ln.split()
        if len(f) == 4 and f[0] == "traffic_over_algorithmic" and f[1] == key and f[3] == cur:
            return float(f[2]) * bytes_per_launch
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(budget_s: float = 12.0):
    """Time the FP64 oracle's Schur apply on the host on a 16^3 x 32 sample."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.dirac import Lattice, WilsonClover
    from paper_2407_08092_amd import synth

    dims = MIXED["dims"]
    with threadpool_limits(1):
        lat = Lattice(dims)
        op = WilsonClover(lat, synth.gauge_field(dims, MIXED["eps"], MIXED["seed_gauge"]), MIXED["c_sw"], MIXED["m0"])
        x = synth.gaussian_complex((lat.Vh, 12), MIXED["seed_vec"])
        n, t0 = 0, time.perf_counter()
        while True:
            x = op.schur(x) / 4.0
            n += 1
            if time.perf_counter() - t0 > budget_s:
                break
        dt = (time.perf_counter() - t0) / n
    gbs = BYTES_APPLY_F64 * lat.Vh / dt / 1e9
    return {"value": round(gbs, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} FP64 Schur applies on 16^3x32 (V/2 = {lat.Vh}), algorithmic FP64 bytes "
                      f"({BYTES_APPLY_F64} B/even site) / mean time {dt * 1e3:.1f} ms; numpy single thread",
            "host_cores_available": len(os.sched_getaffinity(0))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--multi-rhs-only", action="store_true")
    ap.add_argument("--mrhs-only", action="store_true")
    ap.add_argument("--sap-only", action="store_true")
    ap.add_argument("--headline-only", action="store_true")
    ap.add_argument("--batch-only", action="store_true")
    ap.add_argument("--coarse-only", action="store_true")
    ap.add_argument("--coarse-nv", type=int, nargs="+", default=[24, 20])
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path is single-GPU; "
              f"multi-GPU sharding is design only)", file=sys.stderr)
        sys.exit(2)

    if args.coarse_only:
        import torch

        from paper_2407_08092_amd import api

        torch.cuda.set_device(0)
        print(json.dumps({"coarse": coarse_operator(api, torch, torch.device("cuda:0"), args.coarse_nv)}), flush=True)
        return

    if args.sap_only:
        import torch

        from paper_2407_08092_amd import api, synth

        torch.cuda.set_device(0)
        print(json.dumps({"sap": sap_only(api, synth, torch, torch.device("cuda:0"))}), flush=True)
        return

    if args.mrhs_only:
        import torch

        from paper_2407_08092_amd import api, synth

        torch.cuda.set_device(0)
        print(json.dumps({"mrhs_layout": mrhs_only(api, synth, torch, torch.device("cuda:0"))}), flush=True)
        return

    if args.multi_rhs_only or args.batch_only:
        import torch

        from paper_2407_08092_amd import api, synth

        torch.cuda.set_device(0)
        multi, batch = batched(api, synth, torch, torch.device("cuda:0"), solve=args.batch_only)
        print(json.dumps({"multi_rhs": multi, "batched": batch}), flush=True)
        return

    cpu = None if args.no_cpu else cpu_baseline()
    if cpu:
        log(f"cpu baseline {cpu['value']} GB/s")

    import torch

    from paper_2407_08092_amd import api, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = LARGE
    dims = cfg["dims"]
    t0 = time.time()
    lat = api.create_lattice(dims, device=dev)
    U = synth.gauge_field(dims, cfg["eps"], cfg["seed_gauge"], device=dev)
    api.set_gauge(lat, U)
    del U
    torch.cuda.empty_cache()
    api.set_clover(lat, cfg["c_sw"], cfg["m0"])
    vh = lat.Vh
    g = synth.gaussian_complex((2, 12, vh), cfg["seed_vec"])
    x64 = torch.from_numpy(g[0]).to(dev)
    b64 = torch.from_numpy(g[1]).to(dev)
    del g
    lam = api.estimate_lambda_max(lat, 50, x64)
    omega = 0.8 / lam
    x32 = api.convert_parity(lat, x64, torch.complex64)
    b32 = api.convert_parity(lat, b64, torch.complex64)
    y32 = torch.empty_like(x32)
    xs = torch.empty_like(x32)
    log(f"set-up {time.time() - t0:.1f} s, |lambda_max| = {lam:.4f}, omega = {omega:.4f}")

    stream = torch.cuda.current_stream(dev)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        api.apply_schur(lat, x32, y32)
        if ev is not None:
            ev[1].record(stream)
        xs.zero_()
        api.richardson_smooth(lat, xs, b32, SWEEPS, omega)
        if ev is not None:
            ev[2].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    # the library's per-kernel profiler brackets every launch of the first timed step with
    # HIP events on the lattice's stream (an event pair per launch costs a few microseconds,
    # which over the 546 launches of a step would slow every step by ~10%)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        if k == 0:
            api.profile_begin(lat)
        step(evs[k])
        if k == 0:
            prof = api.profile_end(lat)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_start
    t_apply = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps  # ms
    t_sweeps = sum(e[1].elapsed_time(e[2]) for e in evs) / args.steps
    gbs = BYTES_APPLY_F32 * vh / (t_apply * 1e-3) / 1e9
    sweeps_per_s = SWEEPS / (t_sweeps * 1e-3)
    ms_per_step = t_wall / args.steps * 1e3
    log(f"FP32 apply {t_apply:.3f} ms = {gbs:.0f} GB/s; {sweeps_per_s:.1f} sweeps/s")

    # dominant kernel of the timed region
    name, st = max(prof.items(), key=lambda kv: kv[1]["total_ms"])
    ach = st["bytes_per_launch"] / (st["mean_ms"] * 1e-3) / 1e9
    traffic = measured_traffic(name, st["bytes_per_launch"])
    roof = {"bound": "hbm", "kernel": name, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
            "traffic_over_algorithmic": round(traffic / st["bytes_per_launch"], 3) if traffic else None,
            "bytes_per_launch": st["bytes_per_launch"], "mean_ms": round(st["mean_ms"], 4),
            "launches": st["launches"],
            "all_kernels": {k: {"mean_ms": round(v["mean_ms"], 4), "launches": v["launches"],
                                "GBs": round(v["bytes_per_launch"] / (v["mean_ms"] * 1e-3) / 1e9, 1)}
                            for k, v in prof.items()}}

    if args.headline_only:  # profiling run: the timed FP32 step only, its own JSON
        print(json.dumps({"apply_ms": round(t_apply, 4), "apply_GBs": round(gbs, 1),
                          "sweeps_per_s": round(sweeps_per_s, 1), "roofline": roof}), flush=True)
        return

    # the same apply and sweeps as one launch per kernel (no t-chunks): what the chunked
    # launches gain by reading u_o back from the Infinity Cache
    api.set_sweep_chunks(lat, 1)
    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    ev1 = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    for k in range(args.steps):
        step(ev1[k])
    torch.cuda.synchronize()
    api.set_sweep_chunks(lat, 0)
    t1a = sum(e[0].elapsed_time(e[1]) for e in ev1) / args.steps
    t1s = sum(e[1].elapsed_time(e[2]) for e in ev1) / args.steps
    one_launch = {"apply_ms": round(t1a, 4), "apply_GBs": round(BYTES_APPLY_F32 * vh / (t1a * 1e-3) / 1e9, 1),
                  "sweeps_per_s": round(SWEEPS / (t1s * 1e-3), 1)}
    log(f"one launch per kernel (no t-chunks): {one_launch}")

    # the streaming ceiling of each stencil kernel's byte mix on the same fields
    mix = stencil_stream_ceiling(api, torch, lat, x32, xs, b32, y32, args.steps)
    roof["stream_mix_GBs"] = mix
    if "stream_" + name in mix:
        roof["frac_of_stream_mix"] = round(ach / mix["stream_" + name], 4)
    log(f"streaming ceilings of the stencil kernels' byte mix: {mix}")

    # the same FP32 step with 12-real links (third row rebuilt from unitarity)
    U = synth.gauge_field(dims, cfg["eps"], cfg["seed_gauge"], device=dev)
    api.set_gauge(lat, U, link12=True)
    del U
    torch.cuda.empty_cache()
    api.set_clover(lat, cfg["c_sw"], cfg["m0"])
    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    ev12 = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    for k in range(args.steps):
        step(ev12[k])
    torch.cuda.synchronize()
    t12 = sum(e[0].elapsed_time(e[1]) for e in ev12) / args.steps
    s12 = sum(e[1].elapsed_time(e[2]) for e in ev12) / args.steps
    link12 = {"apply_ms": round(t12, 4), "apply_GBs": round(BYTES_APPLY_F32_L12 * vh / (t12 * 1e-3) / 1e9, 1),
              "bytes_per_even_site": BYTES_APPLY_F32_L12, "sweeps_per_s": round(SWEEPS / (s12 * 1e-3), 1)}
    log(f"FP32 12-real links: apply {t12:.3f} ms, {link12['sweeps_per_s']} sweeps/s")

    # 16-bit storage (FP16, BF16) with FP32 arithmetic
    U = synth.gauge_field(dims, cfg["eps"], cfg["seed_gauge"], device=dev)
    api.set_gauge(lat, U, store=(api.DDQ_F64, api.DDQ_F32, api.DDQ_F16, api.DDQ_BF16), link12=True)
    del U
    torch.cuda.empty_cache()
    api.set_clover(lat, cfg["c_sw"], cfg["m0"])
    h16 = {}
    for label, dt, c32 in (("fp16", torch.float16, False), ("bf16", torch.bfloat16, False),
                           ("fp16_clover32", torch.float16, True), ("bf16_clover32", torch.bfloat16, True)):
        api.set_h16_clover(lat, c32)
        bps = BYTES_APPLY_H16_C32 if c32 else BYTES_APPLY_H16
        x16 = api.convert_parity(lat, x64, dt)
        b16 = api.convert_parity(lat, b64, dt)
        y16, xs16 = torch.empty_like(x16), torch.empty_like(x16)

        def step16(ev=None):
            if ev is not None:
                ev[0].record(stream)
            api.apply_schur(lat, x16, y16)
            if ev is not None:
                ev[1].record(stream)
            xs16.zero_()
            api.richardson_smooth(lat, xs16, b16, SWEEPS, omega)
            if ev is not None:
                ev[2].record(stream)

        for _ in range(max(1, args.warmup)):
            step16()
        torch.cuda.synchronize()
        ev16 = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
        for k in range(args.steps):
            step16(ev16[k])
        torch.cuda.synchronize()
        ta = sum(e[0].elapsed_time(e[1]) for e in ev16) / args.steps
        tsw = sum(e[1].elapsed_time(e[2]) for e in ev16) / args.steps
        ref = api.convert_parity(lat, y32, torch.complex128)
        got = api.convert_parity(lat, y16, torch.complex128)
        h16[label] = {"apply_ms": round(ta, 4), "apply_GBs": round(bps * vh / (ta * 1e-3) / 1e9, 1),
                      "bytes_per_even_site": bps, "sweeps_per_s": round(SWEEPS / (tsw * 1e-3), 1),
                      "rel_diff_vs_fp32_apply": float((got - ref).norm() / ref.norm())}
        log(f"{label} storage: apply {ta:.3f} ms, {h16[label]['sweeps_per_s']} sweeps/s")
        del x16, b16, y16, xs16, ref, got
    api.set_h16_clover(lat, False)

    # FP64 apply and sweeps on the same lattice (context)
    y64 = torch.empty_like(x64)
    for _ in range(2):
        api.apply_schur(lat, x64, y64)
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    n64 = max(3, args.steps // 4)
    e0.record(stream)
    for _ in range(n64):
        api.apply_schur(lat, x64, y64)
    e1.record(stream)
    xs64 = torch.zeros_like(x64)
    api.richardson_smooth(lat, xs64, b64, SWEEPS, omega)
    e2.record(stream)
    torch.cuda.synchronize()
    t64 = e0.elapsed_time(e1) / n64
    fp64 = {"apply_ms": round(t64, 4), "apply_GBs": round(BYTES_APPLY_F64 * vh / (t64 * 1e-3) / 1e9, 1),
            "sweeps_per_s": round(SWEEPS / (e1.elapsed_time(e2) * 1e-3), 1),
            "stream_mix_GBs": stencil_stream_ceiling(api, torch, lat, x64, xs64, b64, y64, 5)}
    # SAP(1, 4) sweeps (Alg. 1, 4^4 blocks; block solves in FP64 and in FP32) on the same
    # lattice: the block kernel's live profile and the sweep time
    fp64.update(sap_sweeps(api, synth, torch, lat, dims, cfg["seed_vec"] + 7))
    del y64, xs64, x64, b64
    api.destroy_lattice(lat)
    del lat
    torch.cuda.empty_cache()

    copy = stream_probe(api, torch, dev)
    stream_gbs = max(copy.values())
    log(f"stream copy {stream_gbs:.0f} GB/s")

    mixed = None
    if not args.no_solve:
        mixed = mixed_vs_fp64(api, synth, torch, dev)
    multi, batch = None, None
    if not args.no_batch:
        multi, batch = batched(api, synth, torch, dev)
    coarse = coarse_operator(api, torch, dev, args.coarse_nv)
    share = one_gpu_share(api, synth, torch, dev)

    out = {
        "metric": METRIC, "value": round(gbs, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "odd-even Wilson-clover 48^3x96, eps 0.5, c_sw 1.2, m0 -0.25, t antiperiodic: "
                               "FP32 Schur apply + 20 FP32 Richardson sweeps per step",
                   "dims": list(dims), "even_sites": vh, "sweeps_per_step": SWEEPS, "omega": round(omega, 6)},
        "pct_hbm_peak": round(100 * gbs / HBM_PEAK_GBS, 2),
        "stream_copy_GBs": round(stream_gbs, 1),
        "stream_copy_detail_GBs": {k: round(v, 1) for k, v in copy.items()},
        "pct_of_stream_copy": round(100 * gbs / stream_gbs, 2),
        "schur_apply_ms": round(t_apply, 4),
        "sweeps_per_s": round(sweeps_per_s, 1),
        "t_chunks": "FP32 one-right-hand-side apply and sweeps launched per range of t-slices (13 ranges, "
                    "u_o of a range about 40 MiB, read back from the Infinity Cache); one_launch: the same "
                    "with one launch per kernel",
        "one_launch": one_launch,
        "fp32_link12": link12,
        "storage_16bit": h16,
        "fp64": fp64,
        "mixed_vs_fp64": mixed,
        "multi_rhs": multi,
        "batched": batch,
        "coarse": coarse,
        "one_gpu_share": share,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


MFMA_F32_PEAK_TFLOPS = 157.3


def sap_sweeps(api, synth, torch, lat, dims, seed, nsap=3):
    """SAP(1, 4) sweeps on D x = b (Alg. 1, 4^4 blocks) with FP64 and with FP32 block
    solves: the sweep time and the library profiler's figures of the block kernels."""
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    bf = torch.from_numpy(synth.gaussian_spinor(dims, seed)).to(lat.device)
    xf = torch.zeros_like(bf)
    out = {}
    for label, prec in (("sap_1x4_f64", api.DDQ_F64), ("sap_1x4_f32", api.DDQ_F32)):
        api.sap_smooth(lat, bf, xf, 1, 4, prec=prec)
        torch.cuda.synchronize()
        api.profile_begin(lat)
        e0.record(stream)
        api.sap_smooth(lat, bf, xf, nsap, 4, prec=prec)
        e1.record(stream)
        torch.cuda.synchronize()
        sprof = api.profile_end(lat)
        sap = {"sweep_ms": round(e0.elapsed_time(e1) / nsap, 3),
               "kernels": {k: {"mean_ms": round(v["mean_ms"], 4), "launches": v["launches"],
                               "GBs": round(v["bytes_per_launch"] / (v["mean_ms"] * 1e-3) / 1e9, 1)}
                           for k, v in sprof.items()}}
        out[label] = sap
        log(f"SAP(1, 4) on {'x'.join(map(str, dims))}, {label}: {sap}")
    return out


def sap_only(api, synth, torch, dev):
    """--sap-only: the SAP sweeps of the full run on the 48^3x96 lattice, FP32 block
    solves with 12-real links."""
    cfg = LARGE
    dims = cfg["dims"]
    lat = api.create_lattice(dims, device=dev)
    api.set_gauge(lat, synth.gauge_field(dims, cfg["eps"], cfg["seed_gauge"], device=dev), link12=True)
    api.set_clover(lat, cfg["c_sw"], cfg["m0"])
    out = sap_sweeps(api, synth, torch, lat, dims, cfg["seed_vec"] + 7)
    api.destroy_lattice(lat)
    return out


def one_gpu_share(api, synth, torch, dev, reps=20):
    """The FP32 Schur apply and Richardson sweep on 48^3 x 12: one GPU's share of 48^3 x 96
    split over 8 GPUs in t.  The t wrap-around of this lattice stands in for the halo a
    sharded run would receive (the same bytes per site); no exchange is made."""
    dims = (48, 48, 48, 12)
    lat = api.create_lattice(dims, device=dev)
    api.set_gauge(lat, synth.gauge_field(dims, LARGE["eps"], LARGE["seed_gauge"] + 50, device=dev))
    api.set_clover(lat, LARGE["c_sw"], LARGE["m0"])
    vh = lat.Vh
    g = synth.gaussian_complex((2, 12, vh), LARGE["seed_vec"] + 50)
    x = api.convert_parity(lat, torch.from_numpy(g[0]).to(dev), torch.complex64)
    b = api.convert_parity(lat, torch.from_numpy(g[1]).to(dev), torch.complex64)
    del g
    y = torch.empty_like(x)
    xs = torch.zeros_like(x)
    for _ in range(3):
        api.apply_schur(lat, x, y)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        api.apply_schur(lat, x, y)
    e1.record()
    api.richardson_smooth(lat, xs, b, SWEEPS, 0.1)
    e2.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    out = {"workload": "48^3x12 (one GPU's share of 48^3x96 over 8 GPUs in t), FP32 Schur apply and "
                       "Richardson sweeps, no halo exchange", "dims": list(dims), "even_sites": vh,
           "apply_ms": round(ms, 4), "apply_GBs": round(BYTES_APPLY_F32 * vh / (ms * 1e-3) / 1e9, 1),
           "sweeps_per_s": round(SWEEPS / (e1.elapsed_time(e2) * 1e-3), 1)}
    log(f"one GPU's share 48^3x12: {out}")
    api.destroy_lattice(lat)
    del x, b, y, xs
    torch.cuda.empty_cache()
    return out


def coarse_operator(api, torch, dev, nvs=(24, 20), reps=10):
    """The coarse-grid operator (Sect. 2.3) on the coarsening of 48^3 x 96 by 4^4
    aggregates (12^3 x 24 coarse sites), random FP32 blocks, N_v = 24 and 20, 16 and 64
    right-hand sides.  Algorithmic flops per site: 9 blocks x 8 (2 N_v)^2 per right-hand
    side; algorithmic bytes: the nine FP32 blocks once per group of right-hand sides
    sharing a wave (9 x (2 N_v)^2 x 8 B per site and group), the input vectors once and
    the output once (2 N_v x nrhs x 8 B each per site)."""
    cd = (12, 12, 12, 24)
    vc = 12 * 12 * 12 * 24
    out = {"workload": "coarse operator of 48^3x96 with 4^4 aggregates: 12^3x24 coarse sites, nine "
                       "2N_v x 2N_v FP32 complex blocks per site, random blocks and vectors",
           "coarse_dims": list(cd), "peak_TFLOPs_fp32_mfma": MFMA_F32_PEAK_TFLOPS}
    for nv in nvs:
        n2 = 2 * nv
        g = torch.Generator(device=dev).manual_seed(900 + nv)
        blocks = torch.randn((vc, 9, n2, n2), dtype=torch.complex64, device=dev, generator=g)
        op = api.CoarseOperator(cd, blocks)
        op16 = api.CoarseOperator(cd, blocks, storage=api.DDQ_F16) if nv == 24 else None
        del blocks
        for nrhs in (16, 64):
            v = torch.randn((vc, n2, nrhs), dtype=torch.complex64, device=dev, generator=g)
            y = torch.empty_like(v)
            for _ in range(2):
                op.apply(v, y)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                op.apply(v, y)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            tiles = (nrhs + 15) // 16
            groups = (tiles + 3) // 4  # N_v <= 24: the default groups at most 4 tiles
            flops = 8.0 * n2 * n2 * nrhs * 9 * vc
            nbytes = groups * 9 * n2 * n2 * 8 * vc + 2 * n2 * nrhs * 8 * vc
            tf = flops / (ms * 1e-3) / 1e12
            gbs = nbytes / (ms * 1e-3) / 1e9
            # the matrix-core work actually issued: per site, 9 blocks x (16-row tiles) x
            # (4-wide k-slices) x (16-column right-hand-side tiles) x real products per
            # complex one (Gauss's 3 by default, 4 in the schoolbook form) x 2048 flops of
            # one v_mfma_f32_16x16x4_f32, padding included; its fraction of the FP32 matrix
            # peak cannot exceed 1
            def issued(ms_, products):
                per_site = 9 * ((n2 + 15) // 16) * 2 * ((n2 + 7) // 8) * tiles * products * 2048
                return per_site * vc / (ms_ * 1e-3) / 1e12
            out[f"nv{nv}_rhs{nrhs}"] = {"ms": round(ms, 4), "TFLOPs_algorithmic": round(tf, 1),
                                        "mfma_TFLOPs_issued": round(issued(ms, 3), 1),
                                        "frac_mfma_peak": round(issued(ms, 3) / MFMA_F32_PEAK_TFLOPS, 3),
                                        "GBs": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 3),
                                        "flop_per_byte": round(flops / nbytes, 2)}
            if nrhs == 64:  # the schoolbook form (4 real products) for comparison
                for _ in range(2):
                    op.apply(v, y, product=1)
                torch.cuda.synchronize()
                e0.record()
                for _ in range(reps):
                    op.apply(v, y, product=1)
                e1.record()
                torch.cuda.synchronize()
                ms4 = e0.elapsed_time(e1) / reps
                out[f"nv{nv}_rhs{nrhs}"]["four_products"] = {
                    "ms": round(ms4, 4), "TFLOPs_algorithmic": round(flops / (ms4 * 1e-3) / 1e12, 1),
                    "mfma_TFLOPs_issued": round(issued(ms4, 4), 1),
                    "frac_mfma_peak": round(issued(ms4, 4) / MFMA_F32_PEAK_TFLOPS, 3)}
            if op16 is not None:  # FP16 block storage: half the block bytes, FP32 arithmetic
                for _ in range(2):
                    op16.apply(v, y)
                torch.cuda.synchronize()
                e0.record()
                for _ in range(reps):
                    op16.apply(v, y)
                e1.record()
                torch.cuda.synchronize()
                ms16 = e0.elapsed_time(e1) / reps
                nbytes16 = groups * 9 * n2 * n2 * 4 * vc + 2 * n2 * nrhs * 8 * vc
                out[f"nv{nv}_rhs{nrhs}"]["f16_blocks"] = {
                    "ms": round(ms16, 4), "TFLOPs_algorithmic": round(flops / (ms16 * 1e-3) / 1e12, 1),
                    "mfma_TFLOPs_issued": round(issued(ms16, 3), 1),
                    "frac_mfma_peak": round(issued(ms16, 3) / MFMA_F32_PEAK_TFLOPS, 3),
                    "GBs": round(nbytes16 / (ms16 * 1e-3) / 1e9, 1)}
            log(f"coarse N_v={nv} nrhs={nrhs}: {out[f'nv{nv}_rhs{nrhs}']}")
            del v, y
        del op, op16
        torch.cuda.empty_cache()
    return out


def stencil_stream_ceiling(api, torch, lat, vin, x, b, out, reps):
    """GB/s of the library's streaming-ceiling probe for kernels A, B apply and B
    Richardson: each kernel's algorithmic bytes, layouts, workgroup order and cache
    policies without the neighbour gathers and the arithmetic, timed by the same
    library profiling as the stencil."""
    for k in range(3):
        api.stencil_stream(lat, k, vin, out, x, b)
    torch.cuda.synchronize()
    api.profile_begin(lat)
    for _ in range(max(reps, 5)):
        for k in range(3):
            api.stencil_stream(lat, k, vin, out, x, b)
    torch.cuda.synchronize()
    prof = api.profile_end(lat)
    return {k: round(v["bytes_per_launch"] / (v["mean_ms"] * 1e-3) / 1e9, 1) for k, v in prof.items()}


def stream_probe(api, torch, dev, nbytes=4 << 30, reps=5):
    """Attainable HBM bandwidth: the library's STREAM-style copy of 4 GiB,
    (read + write bytes) / time, plain and with non-temporal accesses."""
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    src.fill_(1)
    out = {}
    for nt in (False, True):
        api.stream_copy(dst, src, nt)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            api.stream_copy(dst, src, nt)
        e1.record()
        torch.cuda.synchronize()
        out["nontemporal" if nt else "plain"] = 2 * nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return out


def mixed_vs_fp64(api, synth, torch, dev):
    cfg = MIXED
    dims = cfg["dims"]
    lat = api.create_lattice(dims, device=dev)
    api.set_gauge(lat, synth.gauge_field(dims, cfg["eps"], cfg["seed_gauge"], device=dev),
                  store=(api.DDQ_F64, api.DDQ_F32, api.DDQ_F16, api.DDQ_BF16))
    api.set_clover(lat, cfg["c_sw"], cfg["m0"])
    b = torch.from_numpy(synth.gaussian_spinor(dims, cfg["seed_vec"])).to(dev)
    v0 = torch.from_numpy(synth.gaussian_complex((12, lat.Vh), cfg["seed_vec"] + 1)).to(dev)
    omega = 0.8 / api.estimate_lambda_max(lat, 50, v0)
    runs = {}
    variants = {
        "fp64_gmres50": dict(inner_prec=api.DDQ_F64, smoother_sweeps=0),
        "fp64_gmres50_rich4": dict(inner_prec=api.DDQ_F64, smoother_sweeps=4),
        "mixed_gmres50": dict(inner_prec=api.DDQ_F32, smoother_sweeps=0),
        "mixed_gmres50_rich4": dict(inner_prec=api.DDQ_F32, smoother_sweeps=4),
        "mixed_gmres50_rich4_fp16": dict(inner_prec=api.DDQ_F32, smoother_sweeps=4, smoother_prec=api.DDQ_F16),
        "mixed_gmres50_rich4_bf16": dict(inner_prec=api.DDQ_F32, smoother_sweeps=4, smoother_prec=api.DDQ_BF16),
        "mixed_gmres50_rich8_fp16": dict(inner_prec=api.DDQ_F32, smoother_sweeps=8, smoother_prec=api.DDQ_F16),
        "mixed_gmres50_rich12_fp16": dict(inner_prec=api.DDQ_F32, smoother_sweeps=12, smoother_prec=api.DDQ_F16),
        "mixed_gmres50_rich12_fp16_cgs1": dict(inner_prec=api.DDQ_F32, smoother_sweeps=12,
                                               smoother_prec=api.DDQ_F16, orth_passes=1),
    }
    for name, kw in variants.items():
        best = None
        for _ in range(2):  # first call warms up and sizes the basis
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info, ok = api.oe_gmres_solve(lat, b, m=50, max_cycles=200, tol=1e-10, omega=omega, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        runs[name] = {"time_s": round(best, 4), "converged": bool(ok), "cycles": info["cycles"],
                      "iters": info["iters"], "applies_f64": info["applies_f64"], "applies_f32": info["applies_lo"],
                      "relres": info["true_relres"]}
        log(f"{name}: {runs[name]}")
    # FGMRES on the full D with the odd-even smoother M_nu (Sect. 2.4.5) as right
    # preconditioner, to the same |b - D x| <= 1e-10 |b|
    full = {}
    for name, kw in {"fgmres50_full_oe3_f64": dict(smoother_sweeps=3, inner_prec=api.DDQ_F64),
                     "fgmres50_full_oe8_f64": dict(smoother_sweeps=8, inner_prec=api.DDQ_F64),
                     "fgmres50_full_oe8_f32": dict(smoother_sweeps=8, inner_prec=api.DDQ_F32),
                     "fgmres50_full_oe16_f32": dict(smoother_sweeps=16, inner_prec=api.DDQ_F32),
                     "fgmres50_full_sap1x4_f64": dict(sap_n=1, sap_m=4, inner_prec=api.DDQ_F64),
                     "fgmres50_full_sap1x4_f32": dict(sap_n=1, sap_m=4, inner_prec=api.DDQ_F32),
                     "fgmres50_full_sap2x4_f32": dict(sap_n=2, sap_m=4, inner_prec=api.DDQ_F32)}.items():
        best = None
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if "sap" in name:
                x, info, ok = api.fgmres_sap_solve(lat, b, m=50, max_cycles=200, tol=1e-10, **kw)
            else:
                x, info, ok = api.fgmres_solve(lat, b, m=50, max_cycles=200, tol=1e-10, omega=omega, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        full[name] = {"time_s": round(best, 4), "converged": bool(ok), "cycles": info["cycles"],
                      "iters": info["iters"], "applies_f64": info["applies_f64"], "applies_f32": info["applies_lo"],
                      "relres": info["true_relres"]}
        log(f"{name}: {full[name]}")
    fp64_best = min(v["time_s"] for k, v in runs.items() if k.startswith("fp64") and v["converged"])
    mixed_best = min(v["time_s"] for k, v in runs.items() if k.startswith("mixed") and v["converged"])
    api.destroy_lattice(lat)
    return {"workload": "16^3x32, eps 0.5, c_sw 1.0, m0 -0.2, Gaussian b, tol 1e-10 (|b - D x| / |b|, FP64)",
            "runs": runs, "fp64_best_s": fp64_best, "mixed_best_s": mixed_best,
            "speedup": round(fp64_best / mixed_best, 3),
            "fgmres_full_oe_smoother": full}


def timed_events(torch, fn, reps=20):
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def mrhs_only(api, synth, torch, dev):
    """Profiling run: only the interleaved-layout stencil on the batching workload's
    24^3 x 48 lattice with 12 right-hand sides."""
    dims, n, seed = BATCH[0]
    lat = api.create_lattice(dims, device=dev)
    api.set_gauge(lat, synth.gauge_field(dims, 0.5, seed, device=dev))
    api.set_clover(lat, 1.0, -0.2)
    x = api.convert_parity(lat, torch.from_numpy(synth.gaussian_complex((n, 12, lat.Vh), 405)).to(dev), torch.complex64)
    return mrhs_layout(api, torch, lat, x, n, lambda fn, reps=20: timed_events(torch, fn, reps))


def mrhs_layout(api, torch, lat, x_planar, n, timed):
    """The interleaved-layout stencil (right-hand sides contiguous per site) on the same
    vectors: apply and Richardson sweep per engine, workgroup order and LDS cap; the
    per-kernel mean durations of the fastest setting from the library's profiler."""
    vh = lat.Vh
    xm = api.mrhs_pack(lat, x_planar)
    ym = torch.empty_like(xm)
    bm = xm.flip(2).contiguous()
    wm = xm.clone()
    bytes_apply = (12 * 5 * n + 144 + 72) * 8 * vh
    bytes_sweep = (12 * 6 * n + 144 + 72) * 8 * vh
    res = {"layout": "[V/2][6][nrhs][2] complex64", "bytes_per_apply": bytes_apply, "bytes_per_sweep": bytes_sweep,
           "settings": {}}
    best = None
    lt = lat.dims[3]
    launches = [(o, lds, 0, st) for st in (0, 1) for o in (1, 0) for lds in (0, 64)] + \
               [(2, lds, ts, st) for st in (0, 1) for ts in sorted({2, 4, lt // 2}) if ts <= lt // 2 for lds in (0, 64)]
    for engine, ename in ((api.DDQ_ENGINE_VALU, "valu"), (api.DDQ_ENGINE_MFMA, "mfma")):
        for order, lds, tsteps, stage in launches:
            api.mrhs_set_launch(lat, order, lds, tsteps, stage)
            ta = timed(lambda: api.mrhs_apply_schur(lat, xm, ym, engine=engine))
            ts = timed(lambda: api.mrhs_richardson_smooth(lat, wm, bm, 1, 0.1, engine=engine))
            key = f"{ename}_order{order}_lds{lds}" + (f"_t{tsteps}" if order == 2 else "") + ("_staged" if stage else "")
            res["settings"][key] = {"apply_ms": round(ta, 4), "apply_GBs": round(bytes_apply / (ta * 1e-3) / 1e9, 1),
                                    "sweep_ms": round(ts, 4)}
            if best is None or ta < best[0]:
                best = (ta, engine, order, lds, tsteps, stage, key)
    ta, engine, order, lds, tsteps, stage, key = best
    api.mrhs_set_launch(lat, order, lds, tsteps, stage)
    api.profile_begin(lat)
    for _ in range(10):
        api.mrhs_apply_schur(lat, xm, ym, engine=engine)
        api.mrhs_richardson_smooth(lat, wm, bm, 1, 0.1, engine=engine)
    torch.cuda.synchronize()
    kstats = api.profile_end(lat)
    api.mrhs_set_launch(lat, 1, 0)
    res.update({"best": key, "apply_ms": round(ta, 4), "apply_GBs": round(bytes_apply / (ta * 1e-3) / 1e9, 1),
                "frac_of_8TBs": round(bytes_apply / (ta * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "kernels": {name: {"mean_ms": round(k["mean_ms"], 4),
                                   "GBs": round(k["bytes_per_launch"] / (k["mean_ms"] * 1e-3) / 1e9, 1),
                                   "frac_of_8TBs": round(k["bytes_per_launch"] / (k["mean_ms"] * 1e-3) / 1e9 /
                                                         HBM_PEAK_GBS, 4)}
                            for name, k in kstats.items()}})
    log(f"mrhs layout: best {key}: {res['apply_ms']} ms = {res['apply_GBs']} GB/s")
    del xm, ym, bm, wm
    return res


def batched(api, synth, torch, dev, solve=True):
    """Multi-right-hand-side apply and (solve) the batched solve of uneven lattices."""
    lats, bs, oms = [], [], []
    for dims, n, seed in BATCH:
        lat = api.create_lattice(dims, device=dev)
        api.set_gauge(lat, synth.gauge_field(dims, 0.5, seed, device=dev), store=(api.DDQ_F64, api.DDQ_F32, api.DDQ_F16))
        api.set_clover(lat, 1.0, -0.2)
        v0 = torch.from_numpy(synth.gaussian_complex((12, lat.Vh), seed + 2000)).to(dev)
        oms.append(0.8 / api.estimate_lambda_max(lat, 50, v0))
        bs.append(torch.stack([torch.from_numpy(synth.gaussian_spinor(dims, seed + 1000 + r)) for r in range(n)]).to(dev))
        lats.append(lat)

    # 12-right-hand-side FP32 apply on 24^3 x 48
    lat, n = lats[0], BATCH[0][1]
    vh = lat.Vh
    best, cands = api.tune_multi_rhs(lat, n, reps=10)
    x = api.convert_parity(lat, torch.from_numpy(synth.gaussian_complex((n, 12, vh), 405)).to(dev), torch.complex64)
    y = torch.empty_like(x)

    def timed(fn, reps=20):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_multi = timed(lambda: api.apply_schur(lat, x, y))
    x1, y1 = x[0].contiguous(), torch.empty_like(x[0])
    t_one = timed(lambda: api.apply_schur(lat, x1, y1))
    bytes_multi = (12 * 5 * n + 144 + 72) * 8 * vh  # 5 spinor passes per rhs; links and clover twice
    planar = {"layout": "planar [nrhs][6][V/2][2] complex64, register-blocked tile", "tile": best,
              "candidates": [(c["nb"], c["waves"], c["xcd_map"], round(c["ms"], 4)) for c in cands],
              "apply_ms": round(t_multi, 4), "apply_GBs": round(bytes_multi / (t_multi * 1e-3) / 1e9, 1),
              "speedup_vs_single_loop": round(n * t_one / t_multi, 3)}
    log(f"multi-rhs planar: {planar['apply_ms']} ms = {planar['apply_GBs']} GB/s, "
        f"x{planar['speedup_vs_single_loop']} vs {n} single applies, tile {best}")
    inter = mrhs_layout(api, torch, lat, x, n, timed)
    # the faster of the two layouts, against the same algorithmic bytes
    if inter["apply_ms"] < planar["apply_ms"]:
        fast = {"layout": "interleaved", "setting": inter["best"], "apply_ms": inter["apply_ms"]}
    else:
        fast = {"layout": "planar", "setting": best, "apply_ms": planar["apply_ms"]}
    gbs = bytes_multi / (fast["apply_ms"] * 1e-3) / 1e9
    fast.update({"apply_GBs": round(gbs, 1), "frac_of_8TBs": round(gbs / HBM_PEAK_GBS, 4),
                 "speedup_vs_single_loop": round(n * t_one / fast["apply_ms"], 3)})
    # the same 12 right-hand sides in FP16 storage (16-bit spinors and 12-real links, FP32
    # arithmetic; up to three right-hand sides per thread): 240 B of spinor passes per
    # right-hand side, 384 B of links and 320 B of 16-bit clover slots per site
    x16 = api.convert_parity(lat, api.convert_parity(lat, x, torch.complex128), torch.float16)
    y16 = torch.empty_like(x16)
    t16 = timed(lambda: api.apply_schur(lat, x16, y16))
    bytes16 = (240 * n + 384 + 320) * vh
    api.apply_schur(lat, x, y)  # the FP32 result to compare with
    ref = api.convert_parity(lat, y, torch.complex128)
    got = api.convert_parity(lat, y16, torch.complex128)
    fp16 = {"apply_ms": round(t16, 4), "apply_GBs": round(bytes16 / (t16 * 1e-3) / 1e9, 1),
            "bytes_per_apply": bytes16, "speedup_vs_fastest_fp32": round(fast["apply_ms"] / t16, 3),
            "rel_diff_vs_fp32": float((got - ref).norm() / ref.norm())}
    log(f"multi-rhs FP16 storage: {fp16['apply_ms']} ms = {fp16['apply_GBs']} GB/s")
    del x16, y16, ref, got
    multi = {"workload": "24^3x48, 12 right-hand sides, FP32 Schur apply", "bytes_per_apply": bytes_multi,
             "single_apply_ms": round(t_one, 4), "best": fast, "planar": planar, "mrhs_layout": inter,
             "fp16_storage": fp16}
    del x, y, x1, y1
    if not solve:
        for lat in lats:
            api.destroy_lattice(lat)
        torch.cuda.empty_cache()
        return multi, None

    # all 24 systems: one batched solve (several preconditioner settings) vs one by one
    batch = api.batch_create(lats, [b.shape[0] for b in bs])
    variants = {}
    for label, nu, sp, op in (("rich4_fp32", 4, api.DDQ_F32, 2), ("rich4_fp16", 4, api.DDQ_F16, 2),
                              ("rich8_fp16", 8, api.DDQ_F16, 2), ("rich12_fp16", 12, api.DDQ_F16, 2),
                              ("rich16_fp16", 16, api.DDQ_F16, 2), ("rich12_fp16_cgs1", 12, api.DDQ_F16, 1),
                              ("rich16_fp16_cgs1", 16, api.DDQ_F16, 1), ("rich16_fp16_cgs1_cycle12", 16, api.DDQ_F16, 1)):
        best = None
        for _ in range(2):  # the first call tunes, sizes and captures
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cyc = "_cycle" in label  # one graph launch per restart cycle of m steps
            m = int(label.split("_cycle")[1]) if cyc else 50
            xs, infos, ok = api.batch_solve(batch, bs, omega=oms, m=m, tol=1e-10, smoother_sweeps=nu, smoother_prec=sp,
                                            orth_passes=op, cycle_graph=cyc)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        variants[label] = {"time_s": round(best, 4), "converged": bool(ok), "cycles": infos[0]["cycles"],
                           "iters": infos[0]["iters"], "max_relres": max(i["true_relres"] for i in infos)}
        log(f"batched {label}: {variants[label]}")
    good = {k: v for k, v in variants.items() if v["converged"]}
    best_label = min(good, key=lambda k: good[k]["time_s"])
    t_batch = good[best_label]["time_s"]
    t_batch4 = variants["rich4_fp32"]["time_s"]
    kw = dict(m=50, tol=1e-10, smoother_sweeps=4)
    seq = {}
    for name, inner, nu in (("mixed", api.DDQ_F32, 4), ("fp64", api.DDQ_F64, 4), ("fp64_plain", api.DDQ_F64, 0)):
        for lat, b, om in zip(lats, bs, oms):  # warm-up: size every basis
            api.oe_gmres_solve(lat, b[0].contiguous(), m=50, tol=1e-10, inner_prec=inner, smoother_sweeps=nu, omega=om)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        worst, conv = 0.0, True
        for lat, b, om in zip(lats, bs, oms):
            for r in range(b.shape[0]):
                _, info, okr = api.oe_gmres_solve(lat, b[r].contiguous(), m=50, tol=1e-10, inner_prec=inner,
                                                  smoother_sweeps=nu, omega=om)
                worst, conv = max(worst, info["true_relres"]), conv and okr
        torch.cuda.synchronize()
        seq[name] = {"time_s": round(time.perf_counter() - t0, 4), "converged": conv, "max_relres": worst}
    out = {"workload": "24^3x48 x 12 rhs + 8^4, 12^4, 16^3x32 x 4 rhs; eps 0.5, c_sw 1.0, m0 -0.2; GMRES(50) with "
                       "a Richardson preconditioner (batched: 4-16 sweeps, FP32 or FP16 storage, CGS2 or one-pass "
                       "Gram-Schmidt; one by one: 4 FP32 sweeps, CGS2); tol 1e-10",
           "systems": len(infos), "batched_s": round(t_batch, 4), "batched_best": best_label,
           "batched_variants": variants, "sequential": seq,
           "speedup_same_settings_vs_sequential_mixed": round(seq["mixed"]["time_s"] / t_batch4, 3),
           "speedup_vs_sequential_mixed": round(seq["mixed"]["time_s"] / t_batch, 3),
           "speedup_vs_sequential_fp64": round(min(seq["fp64"]["time_s"], seq["fp64_plain"]["time_s"]) / t_batch, 3)}
    log(f"batched: {out}")
    api.batch_destroy(batch)
    for lat in lats:
        api.destroy_lattice(lat)
    torch.cuda.empty_cache()
    return multi, out


if __name__ == "__main__":
    main()
