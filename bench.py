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

Default workload: 32x32 open Heisenberg lattice, 3-layer 2D minGRU, d = 128,
4096 Neel-like zero-magnetisation samples (~1.9k connected each), BF16
projections.  The FP32 path is measured on the same model with a smaller batch
(the rate is per site-eval) and reported beside it.
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
    "heisenberg32x32": dict(L=32, nl=3, d=128, B=4096, B_fp32=256, k=3),
    "heisenberg52x52": dict(L=52, nl=4, d=256, B=256, B_fp32=32, k=4),
    "heisenberg20x20": dict(L=20, nl=3, d=128, B=8192, B_fp32=512, k=2),
    "heisenberg10x10": dict(L=10, nl=2, d=64, B=4096, B_fp32=1024, k=1),
}

# HBM traffic of the forward kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE runs,
# scaled by the same counters on a plain device copy of known size; valid only
# for the kernel source it was measured on (its SHA-256 is recorded with it).
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "fwd_kernel_heisenberg32x32_traffic.md")
FWD_SOURCE = os.path.join(ROOT, "paper_2605_13807_amd", "csrc", "psr_fwd.hip")

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


def fwd_source_sha() -> str:
    import hashlib
    with open(FWD_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def recorded_traffic() -> dict | None:
    """Traffic per forward launch from the committed record, if it matches this kernel source."""
    if not os.path.exists(TRAFFIC_RECORD):
        return None
    rec = {}
    with open(TRAFFIC_RECORD) as f:
        for line in f:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                rec[k.strip()] = v.strip().strip("`")
    if rec.get("source_sha256") != fwd_source_sha():
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


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="heisenberg32x32", choices=sorted(WORKLOADS))
    ap.add_argument("--batch", type=int, default=0, help="override the number of samples")
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp32"])
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-sampler", action="store_true", help="skip the sampler measurement")
    ap.add_argument("--no-lru", action="store_true", help="skip the 1D LRU measurement")
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

    W = WORKLOADS[args.workload]
    L, nl, d, k = W["L"], W["nl"], W["d"], W["k"]
    B = args.batch or W["B"]
    N = L * L
    dev = torch.device("cuda:0")
    prec = P.BF16 if args.precision == "bf16" else P.FP32

    def setup(prec_, B_):
        m = P.Model(P.SNAKE_2D, L, L, nl, d, prec_)
        th = torch.from_numpy(I.params(P.param_count(m), d, 1000 + k)).to(dev)
        s_np = I.spins_neel_like(B_, L, L, 2000 + k)
        s = torch.from_numpy(s_np).to(dev)
        H = P.Hamiltonian(P.HEISENBERG, L, L)
        conn = P.connected(H, s)
        M = int(conn["n_conn"].sum().item())
        del conn
        ws_e = P._workspace(m, P.OP_LOCAL_ENERGY, B_, dev, args.chunk)
        ws_b = P._workspace(m, P.OP_BACKWARD, B_, dev)
        return m, th, s, s_np, H, M, ws_e, ws_b

    def step(m, th, s, H, ws_e, ws_b):
        e, st, lp = P.local_energy(m, th, H, s, chunk_seqs=args.chunk, ws=ws_e)
        w = P.vmc_weights(e, st)
        O, lpb, g = P.logpsi_backward(m, th, s, w=w, want_O=True, ws=ws_b)
        return e, st, O, g

    def timed(prec_, B_, steps, warmup):
        m, th, s, s_np, H, M, ws_e, ws_b = setup(prec_, B_)
        for _ in range(warmup):
            step(m, th, s, H, ws_e, ws_b)
        torch.cuda.synchronize()
        P.timing_begin()
        t0 = time.perf_counter()
        out = None
        for i in range(steps):
            out = step(m, th, s, H, ws_e, ws_b)
            torch.cuda.synchronize()
            print(f"# step {i + 1}/{steps} done at {time.perf_counter() - t0:.2f} s", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        fwd_ms, fwd_launches = P.timing_end()
        site_evals = N * (B_ + M) + N * B_
        return dict(m=m, th=th, s=s, s_np=s_np, H=H, M=M, dt=(t1 - t0), steps=steps, fwd_ms=fwd_ms,
                    fwd_launches=fwd_launches, site_evals=site_evals, out=out, B=B_)

    print(f"# workload {args.workload}: {L}x{L}, {nl} layers, d={d}, B={B}, {args.precision}", file=sys.stderr,
          flush=True)
    r = timed(prec, B, args.steps, args.warmup)
    ms_step = 1000.0 * r["dt"] / r["steps"]
    value = r["site_evals"] * r["steps"] / r["dt"]
    print(f"# main: {ms_step:.1f} ms/step, {value:.4e} site-evals/s, connected {r['M']}", file=sys.stderr, flush=True)

    # roofline of the dominant kernel (the fused forward), from the live HIP-event timing
    F = flops_per_site(nl, d)
    fwd_flops = F * N * (B + r["M"]) * r["steps"]       # forward site-evals of the timed steps
    fwd_s = r["fwd_ms"] / 1000.0
    achieved = fwd_flops / fwd_s / 1e12
    peak = PEAK["bf16_tflops"] if prec == P.BF16 else PEAK["fp32_tflops"]
    roofline = {
        "bound": "mfma",
        "kernel": "fwd_kernel",
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

    tr = recorded_traffic()
    if tr is not None:
        roofline["traffic"] = tr["bytes_per_launch"]
        roofline["traffic_sequences_per_launch"] = tr["sequences_per_launch"]

    # FP32 path on the same model (smaller batch; rate per site-eval)
    fp32 = None
    if not args.no_fp32 and prec == P.BF16:
        B32 = min(B, W["B_fp32"])
        r32 = timed(P.FP32, B32, 1, 1)
        v32 = r32["site_evals"] / r32["dt"]
        fp32 = {"value": v32, "samples": B32, "ms_per_step": round(1000.0 * r32["dt"], 2),
                "speedup_bf16_over_fp32": round(value / v32, 3),
                "fwd_tflops": round(F * N * (B32 + r32["M"]) / (r32["fwd_ms"] / 1000.0) / 1e12, 2)}
        print(f"# fp32: {v32:.4e} site-evals/s", file=sys.stderr, flush=True)
        del r32

    # exact autoregressive sampler (the step before the path), timed on its own: one
    # kernel per call, on the current stream, bracketed by events on that stream
    sampler = None
    if not args.no_sampler:
        ms_ = P.Model(P.SNAKE_2D, L, L, nl, d, prec)
        u_ = torch.from_numpy(I.uniforms(B, N, 3000 + k)).to(dev)
        ws_s = P._workspace(ms_, P.OP_SAMPLE, B, dev)
        P.sample(ms_, r["th"], u_, ws=ws_s)
        torch.cuda.synchronize()
        reps = 3
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            P.sample(ms_, r["th"], u_, ws=ws_s)
        e1.record()
        torch.cuda.synchronize()
        ms_call = e0.elapsed_time(e1) / reps
        tfl = F * N * B / (ms_call / 1000.0) / 1e12
        sampler = {"kernel": "sample_kernel", "samples": B, "ms_per_call": round(ms_call, 3),
                   "samples_per_s": round(B / (ms_call / 1000.0), 1),
                   "site_evals_per_s": B * N / (ms_call / 1000.0), "dtype": "f32",
                   "bound": "mfma", "achieved": round(tfl, 2), "peak": PEAK["fp32_tflops"], "unit": "TFLOP/s",
                   "frac": round(tfl / PEAK["fp32_tflops"], 4)}
        print(f"# sampler: {ms_call:.1f} ms per {B} samples", file=sys.stderr, flush=True)
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
        # each call timed on its own (events around it, then a synchronisation), as it runs
        # inside E_loc; calls queued back to back measured up to 28 % slower per launch
        reps, ms_calls = 5, []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            P.lru_logpsi(mL, thL, seqL, ws=wsL)
            e1.record()
            torch.cuda.synchronize()
            ms_calls.append(e0.elapsed_time(e1))
        ms_call = sum(ms_calls) / reps
        fl = lru_flops_per_site(nlL, dL, dhL)
        tfl = fl * nL * BL / (ms_call / 1000.0) / 1e12
        lru = {"kernel": "lru_kernel",
               "workload": f"tfim_chain{nL}: 1D LRU {nlL} layers d={dL} d_h={dhL}, {nsL} samples and their "
                           f"{nL} single-flip configurations ({BL} chains)",
               "chains": BL, "sites": nL, "ms_per_call": round(ms_call, 3),
               "site_evals_per_s": BL * nL / (ms_call / 1000.0), "dtype": "f32",
               "flops_per_site_eval": fl, "bound": "mfma", "achieved": round(tfl, 2),
               "peak": PEAK["fp32_tflops"], "unit": "TFLOP/s", "frac": round(tfl / PEAK["fp32_tflops"], 4)}
        print(f"# lru: {ms_call:.2f} ms per {BL} chains of {nL}", file=sys.stderr, flush=True)
        del wsL, seqL
        # the whole E_loc call on the same 1024 samples (enumeration, both forwards, FP64 combine)
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
        print(f"# lru E_loc: {ms_e:.2f} ms per {nsL} samples", file=sys.stderr, flush=True)

    # CPU oracle baseline on a bounded sample, and the E_loc error on that sample
    cpu = None
    err = None
    if not args.no_cpu:
        from oracle import grad as OG
        from oracle import hamiltonian as OH
        from oracle import model as OM
        om = OM.Model("snake2d", L, L, nl, d)
        th_np = r["th"].cpu().numpy()
        oh = OH.Hamiltonian("heisenberg", L, L)
        n_s = 1
        sub = r["s_np"][:n_s]
        threads = torch.get_num_threads()
        t0 = time.perf_counter()
        e_ref = OH.local_energy(lambda c: OM.logpsi(th_np, c, om), oh, sub)
        t_fwd = time.perf_counter() - t0
        conn = OH.connected(oh, sub)
        m_sub = int(conn["n_conn"].sum())
        t1 = time.perf_counter()
        OG.per_sample_grad(th_np, sub, om)
        t_bwd = time.perf_counter() - t1
        cpu_site_evals = N * (n_s + m_sub) + N * n_s
        cpu = {"value": cpu_site_evals / (t_fwd + t_bwd), "unit": "site-evals/s", "cores": threads,
               "kind": "oracle",
               "sample": f"{n_s} sample(s) of the workload with all {m_sub} connected configurations "
                         f"(float64 numpy forward) + 1 per-sample gradient (float64 torch autograd); "
                         f"{t_fwd + t_bwd:.1f} s"}
        e_gpu = r["out"][0][:n_s].cpu().numpy()

        def rel(e):
            return float(np.max(np.abs(e - e_ref) / np.maximum(np.abs(e_ref), 1.0)))

        err = {"eloc_rel_err_vs_fp64_oracle": rel(e_gpu), "samples_checked": n_s}
        if prec == P.BF16:
            # the same sample through the oracle's bfloat16 reading: how much of the
            # error above is the precision's (the GPU follows the reading)
            e_rd = OH.local_energy(lambda c: OM.logpsi(th_np, c, om, bf16=True), oh, sub)
            err["eloc_rel_err_bf16_reading_vs_fp64"] = rel(e_rd)
            err["eloc_rel_err_vs_bf16_reading"] = float(
                np.max(np.abs(e_gpu - e_rd) / np.maximum(np.abs(e_rd), 1.0)))
            # the FP32 path on the same sample
            m32 = P.Model(P.SNAKE_2D, L, L, nl, d, P.FP32)
            e32, _, _ = P.local_energy(m32, r["th"], r["H"], r["s"][:n_s])
            err["eloc_rel_err_fp32_path_vs_fp64"] = rel(e32.cpu().numpy())
        print(f"# cpu oracle: {cpu['value']:.4e} site-evals/s ({t_fwd + t_bwd:.1f} s)", file=sys.stderr, flush=True)

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
        "dtype": "bf16" if prec == P.BF16 else "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: open Heisenberg {L}x{L}, 2D minGRU {nl} layers d={d}, "
                               f"{B} Neel-like samples, all bond-exchange connected configurations "
                               f"({r['M']} total), E_loc + per-sample gradients",
                   "samples": B, "connected": r["M"], "sites": N, "chunk_seqs": args.chunk,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp32_path": fp32,
        "sampler": sampler,
        "lru": lru,
        "error": err,
    }
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
