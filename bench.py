#!/usr/bin/env python3
"""Benchmark of the PSR-NQS hot path on one MI355X.

One step = the whole hot path over one batch of synthetic samples:
  pack spins -> connected configurations (Heisenberg, Marshall basis) ->
  log psi of the samples and of every connected configuration (streamed in
  chunks) -> E_loc and its FP64 mean / variance -> VMC weights ->
  per-sample gradients O_s (reverse-scan adjoint with checkpoints) -> FP64
  gradient estimate g = (2/B) sum (E_loc - mean) O_s.

Metric: site-evals/s of log psi forward + backward, i.e.
  N * (samples + connected configurations)  [forward]
+ N * samples                               [backward]
per second of wall time of the timed steps (inputs resident in HBM).

Default workload: 52x52 open Heisenberg lattice, 4-layer 2D minGRU, d = 256,
256 Neel-like zero-magnetisation samples (~5.3k connected each).  The forward
runs on the BF16 matrix cores with split operands (hi + lo; three products per
projection); the backward runs in FP32.  Beside it: the FP32 path on the same
model (a smaller batch: the rate is per site-eval), the errors against the
float64 oracle (stored oracle local energies of the first samples, log psi of
64 samples, one gradient row), the FP16-split path's error, the oracle timed on
the host, the sampler, the 1D LRU and the 32x32 workload.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: lattice side, layers, d, samples, FP32-comparison samples, seed index
    "heisenberg52x52": dict(L=52, nl=4, d=256, B=256, B_fp32=8, k=4),
    "heisenberg32x32": dict(L=32, nl=3, d=128, B=4096, B_fp32=256, k=3),
    "heisenberg20x20": dict(L=20, nl=3, d=128, B=8192, B_fp32=512, k=2),
    "heisenberg10x10": dict(L=10, nl=2, d=64, B=4096, B_fp32=1024, k=1),
}
GOLDEN = os.path.join(ROOT, "tests", "golden")

# HBM traffic of the forward kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE runs,
# scaled by the same counters on a plain device copy of known size; valid only
# for the kernel source it was measured on (its SHA-256 is recorded with it).
# The split paths at d = 128 and 256 run the units-split kernel (psr_fwd_split.hip).
CSRC = os.path.join(ROOT, "paper_2605_13807_amd", "csrc")
TRAFFIC = {
    "heisenberg52x52": (os.path.join(ROOT, "profiles", "fwd_split_kernel_heisenberg52x52_traffic.md"),
                        ["psr_fwd_split.hip", "psr_fwd_common.h"]),
    "heisenberg32x32": (os.path.join(ROOT, "profiles", "fwd_split_kernel_heisenberg32x32_traffic.md"),
                        ["psr_fwd_split.hip", "psr_fwd_common.h"]),
}

PEAK = {  # MI355X datasheet peaks (dense)
    "bf16_tflops": 2500.0,
    "fp32_tflops": 157.3,
    "hbm_gbs": 8000.0,
}


def flops_per_site(nl: int, d: int) -> float:
    """Algorithmic MFMA flops of one site-eval forward: 2 * (2 d^2 + 5 d^2 (nl-1) + 2 d)."""
    return 2.0 * (2 * d * d + 5 * d * d * (nl - 1) + 2 * d)


def lru_flops_per_site(nl: int, d: int, dh: int) -> float:
    """Dense flops of one site of the 1D LRU: per layer the drive [B_re; B_im] x (2 dh x d),
    the output map [C_re | C_im] (d x 2 dh) and the GLU's two projections (2 d x d), plus the head."""
    return float(nl * (2 * (2 * dh * d) + 2 * (d * 2 * dh) + 2 * (2 * d * d)) + 2 * d)


def fwd_source_sha(files) -> str:
    """SHA-256 over the forward kernel's source files (in the order given)."""
    import hashlib
    h = hashlib.sha256()
    for name in files:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic(workload: str) -> dict | None:
    """Traffic per forward launch from the committed record, if it matches this kernel source."""
    if workload not in TRAFFIC or not os.path.exists(TRAFFIC[workload][0]):
        return None
    record, files = TRAFFIC[workload]
    rec = {}
    with open(record) as f:
        for line in f:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                rec[k.strip()] = v.strip().strip("`")
    if rec.get("source_sha256") != fwd_source_sha(files):
        return None
    return {"bytes_per_launch": float(rec["hbm_bytes_per_launch"]),
            "fetch_bytes_per_launch": float(rec["fetch_bytes_per_launch"]),
            "write_bytes_per_launch": float(rec["write_bytes_per_launch"]),
            "sequences_per_launch": int(rec["sequences_per_launch"])}


def copy_calibration() -> int:
    """A plain 1 GiB device-to-device copy: the reference that FETCH_SIZE / WRITE_SIZE are scaled by."""
    import torch
    n = 1 << 28
    x = torch.ones(n, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 4}))
    return 0


def golden(workload: str):
    """Stored float64 oracle values (tests/golden/gen_fullsize_eloc.py): n_conn, log psi, E_loc per sample."""
    path = os.path.join(GOLDEN, f"{workload}_oracle_eloc.txt")
    if not os.path.exists(path):
        return None
    import numpy as np
    rows = [ln.split() for ln in open(path) if not ln.startswith("#")]
    return (np.array([int(r[1]) for r in rows]), np.array([float(r[2]) for r in rows]),
            np.array([float(r[3]) for r in rows]))


def host_cpu() -> dict:
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_count": os.cpu_count(), "model": model}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="heisenberg52x52", choices=sorted(WORKLOADS))
    ap.add_argument("--batch", type=int, default=0, help="override the number of samples")
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp16", "fp32"])
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-sampler", action="store_true", help="skip the sampler measurement")
    ap.add_argument("--no-lru", action="store_true", help="skip the 1D LRU measurement")
    ap.add_argument("--no-extra", action="store_true", help="skip the 32x32 workload leg")
    ap.add_argument("--chunk", type=int, default=32768)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (reference for the HBM traffic counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration()

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: samples shard across GPUs with no "
                                   "communication in the hot path, which a single GPU cannot exercise",
                          "n_gpus": args.gpus}))
        return 2

    import numpy as np
    import torch

    import paper_2605_13807_amd as P
    import psr_inputs as I

    dev = torch.device("cuda:0")
    PREC = {"bf16": P.BF16, "fp16": P.FP16, "fp32": P.FP32}
    prec = PREC[args.precision]

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    def setup(W, prec_, B_):
        L, nl, d, k = W["L"], W["nl"], W["d"], W["k"]
        m = P.Model(P.SNAKE_2D, L, L, nl, d, prec_)
        th = torch.from_numpy(I.params(P.param_count(m), d, 1000 + k)).to(dev)
        s_np = I.spins_neel_like(B_, L, L, 2000 + k)
        s = torch.from_numpy(s_np).to(dev)
        H = P.Hamiltonian(P.HEISENBERG, L, L)
        M = int(P.connected(H, s)["n_conn"].sum().item())
        ws_e = P._workspace(m, P.OP_LOCAL_ENERGY, B_, dev, args.chunk)
        ws_b = P._workspace(m, P.OP_BACKWARD, B_, dev)
        return m, th, s, s_np, H, M, ws_e, ws_b

    def step(m, th, s, H, ws_e, ws_b):
        e, st, lp = P.local_energy(m, th, H, s, chunk_seqs=args.chunk, ws=ws_e)
        w = P.vmc_weights(e, st)
        O, lpb, g = P.logpsi_backward(m, th, s, w=w, want_O=True, ws=ws_b)
        return e, st, O, g, lp

    def timed(W, prec_, B_, steps, warmup, label):
        L = W["L"]
        N = L * L
        m, th, s, s_np, H, M, ws_e, ws_b = setup(W, prec_, B_)
        t0 = time.perf_counter()
        for i in range(warmup):
            step(m, th, s, H, ws_e, ws_b)
            torch.cuda.synchronize()
            log(f"# {label}: warmup {i + 1}/{warmup} done at {time.perf_counter() - t0:.2f} s")
        torch.cuda.synchronize()
        P.timing_begin()
        t0 = time.perf_counter()
        out = None
        for i in range(steps):
            out = step(m, th, s, H, ws_e, ws_b)
            torch.cuda.synchronize()
            log(f"# {label}: step {i + 1}/{steps} done at {time.perf_counter() - t0:.2f} s")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        fwd_ms, fwd_launches = P.timing_end()
        site_evals = N * (B_ + M) + N * B_
        return dict(m=m, th=th, s=s, s_np=s_np, H=H, M=M, dt=(t1 - t0), steps=steps, fwd_ms=fwd_ms,
                    fwd_launches=fwd_launches, site_evals=site_evals, out=out, B=B_)

    def roofline_of(W, r, prec_, workload):
        L, nl, d = W["L"], W["nl"], W["d"]
        N = L * L
        F = flops_per_site(nl, d)
        fwd_flops = F * N * (r["B"] + r["M"]) * r["steps"]   # forward site-evals of the timed steps
        fwd_s = r["fwd_ms"] / 1000.0
        achieved = fwd_flops / fwd_s / 1e12
        peak = PEAK["fp32_tflops"] if prec_ == P.FP32 else PEAK["bf16_tflops"]
        rf = {
            "bound": "mfma",
            "kernel": "fwd_split_kernel" if (prec_ != P.FP32 and d >= 128) else "fwd_kernel",
            "achieved": round(achieved, 2),
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": None,
            "traffic_note": "HBM bytes per forward launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated); "
                            "null when the kernel source differs from the one profiled",
            "launches": r["fwd_launches"],
            "avg_launch_ms": round(r["fwd_ms"] / max(1, r["fwd_launches"]), 4),
            "flops_per_site_eval": F,
            "fwd_share_of_step": round(fwd_s / r["dt"], 4),
        }
        if prec_ != P.FP32:
            # each projection is three 16-bit matrix products (hi*hi + lo*hi + hi*lo)
            rf["mfma_products_per_projection"] = 3
            rf["issued_mfma_frac"] = round(3 * achieved / peak, 4)
        tr = recorded_traffic(workload) if prec_ == P.BF16 else None
        if tr is not None:
            rf["traffic"] = tr["bytes_per_launch"]
            rf["traffic_sequences_per_launch"] = tr["sequences_per_launch"]
        return rf

    W = WORKLOADS[args.workload]
    L, nl, d, k = W["L"], W["nl"], W["d"], W["k"]
    B = args.batch or W["B"]
    N = L * L
    log(f"# workload {args.workload}: {L}x{L}, {nl} layers, d={d}, B={B}, {args.precision}")
    r = timed(W, prec, B, args.steps, args.warmup, "main")
    ms_step = 1000.0 * r["dt"] / r["steps"]
    value = r["site_evals"] * r["steps"] / r["dt"]
    log(f"# main: {ms_step:.1f} ms/step, {value:.4e} site-evals/s, connected {r['M']}")
    roofline = roofline_of(W, r, prec, args.workload)

    # errors against the float64 oracle: stored local energies and log psi of the first
    # samples (tests/golden/gen_fullsize_eloc.py), on the main run's own E_loc
    err = None
    gold = golden(args.workload)
    e_main = r["out"][0].cpu().numpy()
    if gold is not None:
        n_g, lp_g, e_g = gold
        n_e = int(np.sum(np.isfinite(e_g)))
        n_e = min(n_e, B)
        rel = np.abs(e_main[:n_e] - e_g[:n_e]) / np.maximum(np.abs(e_g[:n_e]), 1.0)
        n_l = min(len(lp_g), B)
        lp_gpu = P.logpsi(r["m"], r["th"], r["s"][:n_l]).double().cpu().numpy()
        err = {"reference": "float64 oracle (stored values, tests/golden)",
               "eloc_samples": n_e,
               "eloc_rel_err_max": float(rel.max()),
               "eloc_mean_rel_err": float(abs(e_main[:n_e].mean() - e_g[:n_e].mean()) / abs(e_g[:n_e].mean())),
               "logpsi_samples": n_l,
               "logpsi_abs_err_max": float(np.abs(lp_gpu - lp_g[:n_l]).max()),
               "logpsi_abs": float(np.abs(lp_g[:n_l]).max())}
        if prec != P.FP16:
            # the FP16-split path (~22-bit operands) on the same samples
            m16 = P.Model(P.SNAKE_2D, L, L, nl, d, P.FP16)
            e16, _, _ = P.local_energy(m16, r["th"], r["H"], r["s"][:n_e])
            lp16 = P.logpsi(m16, r["th"], r["s"][:n_l]).double().cpu().numpy()
            e16 = e16.cpu().numpy()
            err["fp16_split_eloc_rel_err_max"] = float(
                (np.abs(e16 - e_g[:n_e]) / np.maximum(np.abs(e_g[:n_e]), 1.0)).max())
            err["fp16_split_logpsi_abs_err_max"] = float(np.abs(lp16 - lp_g[:n_l]).max())
        log(f"# error: {err}")

    # FP32 path on the same model (smaller batch; rate per site-eval)
    fp32 = None
    if not args.no_fp32 and prec != P.FP32:
        B32 = min(B, W["B_fp32"])
        r32 = timed(W, P.FP32, B32, 1, 1, "fp32")
        v32 = r32["site_evals"] / r32["dt"]
        F = flops_per_site(nl, d)
        fp32 = {"value": v32, "samples": B32, "ms_per_step": round(1000.0 * r32["dt"], 2),
                "speedup_over_fp32": round(value / v32, 3),
                "fwd_tflops": round(F * N * (B32 + r32["M"]) / (r32["fwd_ms"] / 1000.0) / 1e12, 2)}
        if gold is not None:
            e32 = r32["out"][0].cpu().numpy()
            n32 = min(len(e32), int(np.sum(np.isfinite(gold[2]))))
            fp32["eloc_rel_err_max"] = float(
                (np.abs(e32[:n32] - gold[2][:n32]) / np.maximum(np.abs(gold[2][:n32]), 1.0)).max())
        log(f"# fp32: {v32:.4e} site-evals/s")
        del r32

    # the 32x32 workload (3 layers, d = 128), one step of 1024 samples
    extra = None
    if not args.no_extra and args.workload != "heisenberg32x32":
        W2 = WORKLOADS["heisenberg32x32"]
        r2 = timed(W2, prec, 1024, 1, 1, "32x32")
        v2 = r2["site_evals"] / r2["dt"]
        rf2 = roofline_of(W2, r2, prec, "heisenberg32x32")
        extra = {"workload": "heisenberg32x32: open Heisenberg 32x32, 2D minGRU 3 layers d=128, 1024 Neel-like "
                             "samples with all bond-exchange connected configurations",
                 "value": v2, "ms_per_step": round(1000.0 * r2["dt"], 2), "connected": r2["M"],
                 "roofline": rf2}
        g2 = golden("heisenberg32x32")
        if g2 is not None:
            e2 = r2["out"][0].cpu().numpy()[:64]
            extra["eloc_rel_err_max_64"] = float((np.abs(e2 - g2[2][:64]) / np.maximum(np.abs(g2[2][:64]), 1.0)).max())
        log(f"# 32x32: {v2:.4e} site-evals/s")
        del r2

    # exact autoregressive sampler (the step before the path), timed on its own: one
    # kernel per call, on the current stream, bracketed by events on that stream
    sampler = None
    if not args.no_sampler:
        ms_ = P.Model(P.SNAKE_2D, L, L, nl, d, prec)
        u_ = torch.from_numpy(I.uniforms(B, N, 3000 + k)).to(dev)
        ws_s = P._workspace(ms_, P.OP_SAMPLE, B, dev)
        P.sample(ms_, r["th"], u_, ws=ws_s)
        torch.cuda.synchronize()
        reps = 2
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            P.sample(ms_, r["th"], u_, ws=ws_s)
        e1.record()
        torch.cuda.synchronize()
        ms_call = e0.elapsed_time(e1) / reps
        F = flops_per_site(nl, d)
        tfl = F * N * B / (ms_call / 1000.0) / 1e12
        sampler = {"kernel": "sample_kernel", "samples": B, "ms_per_call": round(ms_call, 3),
                   "samples_per_s": round(B / (ms_call / 1000.0), 1),
                   "site_evals_per_s": B * N / (ms_call / 1000.0), "dtype": "f32",
                   "bound": "mfma", "achieved": round(tfl, 2), "peak": PEAK["fp32_tflops"], "unit": "TFLOP/s",
                   "frac": round(tfl / PEAK["fp32_tflops"], 4)}
        log(f"# sampler: {ms_call:.1f} ms per {B} samples")
        del ws_s

    # the 1D LRU ansatz of Table I (3 layers, d = d_h = 64) at N = 256: log psi of the
    # E_loc batch of 1024 samples with their 256 single-flip TFIM configurations each,
    # one kernel per call on the current stream, bracketed by events on that stream
    lru = None
    if not args.no_lru:
        nL, nlL, dL, dhL, nsL = 256, 3, 64, 64, 1024
        mL = P.LruModel(nL, nlL, dL, dhL)
        thL = torch.from_numpy(I.params(P.lru_param_count(mL), dL, 3007)).to(dev)
        sL = torch.from_numpy(I.spins_bernoulli(nsL, nL, 4007)).to(dev)
        cL = P.connected(P.Hamiltonian(P.TFIM, nL, 1, J=1.0, h=1.0), sL, configs=True)
        seqL = torch.cat([sL, cL["conn"].reshape(-1, nL)]).contiguous()
        del cL
        BL = seqL.shape[0]
        wsL = torch.empty(P.lru_workspace_bytes(mL, BL), dtype=torch.uint8, device=dev)
        P.lru_logpsi(mL, thL, seqL, ws=wsL)
        torch.cuda.synchronize()
        reps = 3
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            P.lru_logpsi(mL, thL, seqL, ws=wsL)
        e1.record()
        torch.cuda.synchronize()
        ms_call = e0.elapsed_time(e1) / reps
        fl = lru_flops_per_site(nlL, dL, dhL)
        tfl = fl * nL * BL / (ms_call / 1000.0) / 1e12
        lru = {"kernel": "lru_kernel",
               "workload": f"tfim_chain{nL}: 1D LRU {nlL} layers d={dL} d_h={dhL}, {nsL} samples and their "
                           f"{nL} single-flip configurations ({BL} chains), launches back to back",
               "chains": BL, "sites": nL, "ms_per_call": round(ms_call, 3),
               "site_evals_per_s": BL * nL / (ms_call / 1000.0), "dtype": "f32",
               "flops_per_site_eval": fl, "bound": "mfma", "achieved": round(tfl, 2),
               "peak": PEAK["fp32_tflops"], "unit": "TFLOP/s", "frac": round(tfl / PEAK["fp32_tflops"], 4)}
        log(f"# lru: {ms_call:.2f} ms per {BL} chains of {nL}")
        del wsL, seqL
        HL = P.Hamiltonian(P.TFIM, nL, 1, J=1.0, h=1.0)
        P.lru_local_energy(mL, thL, HL, sL)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            P.lru_local_energy(mL, thL, HL, sL)
        e1.record()
        torch.cuda.synchronize()
        ms_e = e0.elapsed_time(e1) / 3
        lru["eloc_ms_per_call"] = round(ms_e, 3)
        lru["eloc_site_evals_per_s"] = (nsL * (nL + 1)) * nL / (ms_e / 1000.0)
        log(f"# lru E_loc: {ms_e:.2f} ms per {nsL} samples")
        # a whole VMC training step of Table I's model at N = 256 (exact sampling, E_loc,
        # per-sample backward, FP64 estimator, Adam), the quantity Table I reports per step
        from paper_2605_13807_amd.vmc import vmc
        thV = thL.clone()
        vmc(mL, HL, thV, steps=1, batch=nsL, lr=1e-3, seed=11)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        vmc(mL, HL, thV, steps=3, batch=nsL, lr=1e-3, seed=12)
        torch.cuda.synchronize()
        ms_v = 1000.0 * (time.perf_counter() - t0) / 3
        lru["vmc_step_ms"] = round(ms_v, 2)
        lru["vmc_step_note"] = ("one training step at N = 256, 1024 samples: sampler, E_loc, backward, estimator, "
                                "Adam (Table I: 900 ms per step on an H100, context)")
        log(f"# lru VMC step: {ms_v:.1f} ms")

    # CPU baseline: the float64 oracle on a bounded sample of the workload (the first
    # sample and as many of its connected configurations as fit in about 15 s, then
    # that sample's gradient by float64 autograd); the gradient also gives the GPU
    # path's gradient error on that sample
    cpu = None
    if not args.no_cpu:
        from oracle import grad as OG
        from oracle import hamiltonian as OH
        from oracle import model as OM
        om = OM.Model("snake2d", L, L, nl, d)
        th_np = r["th"].cpu().numpy()
        sub = r["s_np"][:1]
        conn = OH.connected(OH.Hamiltonian("heisenberg", L, L), sub)
        flips = OH.apply_flips(sub, conn)
        threads = torch.get_num_threads()
        t0 = time.perf_counter()
        OM.logpsi(th_np, sub, om)
        n_done, step_ = 0, 8
        while n_done < flips.shape[0] and time.perf_counter() - t0 < 15.0:
            OM.logpsi(th_np, flips[n_done: n_done + step_], om)
            n_done += min(step_, flips.shape[0] - n_done)
        t_fwd = time.perf_counter() - t0
        t1 = time.perf_counter()
        _, O_ref = OG.per_sample_grad(th_np, sub, om)
        t_bwd = time.perf_counter() - t1
        cpu_site_evals = N * (1 + n_done) + N
        hc = host_cpu()
        cpu = {"value": cpu_site_evals / (t_fwd + t_bwd), "unit": "site-evals/s", "cores": threads,
               "kind": "oracle", "host_cpu_count": hc["cpu_count"], "host_cpu_model": hc["model"],
               "sample": f"1 sample of the workload and {n_done} of its {flips.shape[0]} connected configurations "
                         f"(float64 numpy forward, {t_fwd:.1f} s) + its gradient (float64 torch autograd, "
                         f"{t_bwd:.1f} s), {threads} threads"}
        O_gpu = r["out"][2][0].double().cpu().numpy()
        gerr = float(np.linalg.norm(O_gpu - O_ref[0]) / np.linalg.norm(O_ref[0]))
        if err is None:
            err = {}
        err["grad_rel_err_sample0"] = gerr
        log(f"# cpu oracle: {cpu['value']:.4e} site-evals/s ({t_fwd + t_bwd:.1f} s); grad rel err {gerr:.2e}")

    dtype = {P.BF16: "bf16 (split hi+lo operands, 3 products)", P.FP16: "fp16 (split hi+lo operands, 3 products)",
             P.FP32: "f32"}[prec]
    line = {
        "metric": "site-evals/s for log psi fwd+bwd (bf16 vs fp32, same GPU) at stated E_loc error",
        "value": value,
        "unit": "site-evals/s",
        "n_gpus": 1,
        "steps": r["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: open Heisenberg {L}x{L}, 2D minGRU {nl} layers d={d}, "
                               f"{B} Neel-like samples, all bond-exchange connected configurations "
                               f"({r['M']} total), E_loc (forward in {args.precision}) + per-sample gradients "
                               f"(FP32 backward)",
                   "samples": B, "connected": r["M"], "sites": N, "chunk_seqs": args.chunk,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "error": err,
        "fp32_path": fp32,
        "workload_32x32": extra,
        "sampler": sampler,
        "lru": lru,
    }
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
