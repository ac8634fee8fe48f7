#!/usr/bin/env python3
"""Benchmark of the local-energy + VMC-gradient step on one MI355X.

One step = nqs_energy_grad on one batch: sample forward, enumeration and
matrix elements of every connected configuration, the MFMA forward on all of
them, the FP64 ratio-and-reduce, the weighted energy and the hand backward.
Prints one JSON line (see the keys below); diagnostics go to stderr.

Workload (default): 60 qubits (30 spatial orbitals, 15 up + 15 down
electrons) Jordan-Wigner Hamiltonian from the seeded molecular-like integral
generator (K ~ 1.19e6 merged Pauli strings), 65536 sector-uniform samples
reduced to unique samples with count weights, masked network L = 4, h = 1024,
BF16 GEMMs with FP32 accumulation and FP64 sums.  The plain FP32 GPU path is
timed on a prefix of the same samples, and the FP64 oracle on a few samples
(the CPU baseline).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS_TFLOPS = {"bf16": 2500.0, "bf16x3": 2500.0, "fp32": 157.3, "fp64": 78.6}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4", help="c1..c4, c5a..c5d")
    ap.add_argument("--batch", type=int, default=None, help="override the batch (diagnostic runs)")
    ap.add_argument("--precision", default=None, help="override the network arithmetic")
    ap.add_argument("--fp32-prefix", type=int, default=1024)
    ap.add_argument("--cpu-samples", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--chunk", type=int, default=0, help="samples per chunk (0 = plan default)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build evaluates one GPU's share of the batch on a single MI355X; "
              "multi-GPU runs are not part of it (see DESIGN.md, sharding).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2208_05637_amd as nqs
    from gen import config_inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    t = time.time()
    terms, params_np, samples, weights, cfg = config_inputs(args.workload, batch=args.batch)
    prec = args.precision or cfg["precision"]
    log(f"inputs: n={cfg['n']} B={len(samples)} unique samples, {time.time() - t:.1f}s")
    ctx = nqs.Context(0)
    H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
    K = H.K
    B = len(samples)
    plan = nqs.Plan(ctx, H, cfg["L"], cfg["h"], cfg["n_up"], cfg["n_dn"], prec, max_batch=B,
                    dedup=cfg["dedup"], chunk_samples=args.chunk)
    log(f"K={K} G={H.G} entries/sample={plan.entries_per_sample} chunk={plan.chunk_samples} "
        f"dedup={plan.dedup} workspace={plan.workspace_size(B) / 2**30:.2f} GiB")
    dev = ctx.device
    params = torch.from_numpy(params_np).to(dev)
    x = torch.from_numpy(samples.view(np.int64)).to(dev)
    w = torch.from_numpy(weights).to(dev)
    eloc = torch.empty((B, 2), dtype=torch.float64, device=dev)
    energy = torch.empty(3, dtype=torch.float64, device=dev)
    grad = torch.empty(plan.n_params, dtype=torch.float64, device=dev)
    plan.workspace(B)

    for i in range(args.warmup):
        t = time.time()
        nqs.energy_grad(plan, params, x, w, eloc=eloc, energy=energy, grad=grad)
        torch.cuda.synchronize()
        log(f"warmup step {i}: {time.time() - t:.2f}s")
    if nqs.device_status(plan):
        raise RuntimeError("device error flag after warm-up")

    plan.profile(True)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(ctx.stream)
    for i in range(args.steps):
        nqs.energy_grad(plan, params, x, w, eloc=eloc, energy=energy, grad=grad)
    ev1.record(ctx.stream)
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    ms_step = ev0.elapsed_time(ev1) / args.steps
    eloc_ms = prof["eloc_ms"] / max(prof["calls"], 1)
    value = B * K / (eloc_ms / 1e3)
    log(f"step {ms_step:.1f} ms, local energy {eloc_ms:.1f} ms, E = {energy[0].item():.10f}")
    fwd_ms_launch = prof["forward_ms"] / max(prof["forward_launches"], 1)
    achieved = prof["forward_flops"] / (prof["forward_ms"] / 1e3) / 1e12
    executed = prof["forward_flops_executed"] / (prof["forward_ms"] / 1e3) / 1e12
    peak = PEAKS_TFLOPS[prec]
    log(f"forward kernel: {prof['forward_launches']} launches, {fwd_ms_launch:.2f} ms/launch, "
        f"{achieved:.1f} TFLOP/s algorithmic, {executed:.1f} TFLOP/s issued (peak {peak})")

    out = {
        "metric": "E_loc samples*terms/s (BF16 network, FP64 sums) + VMC step ms",
        "value": value,
        "unit": "samples*terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {cfg['n']} qubits ({cfg['N']} orbitals, {cfg['n_up']}+{cfg['n_dn']} "
                        f"electrons), K={K} Pauli strings, G={H.G} flips, B={B} unique samples "
                        f"(count weights), masked MLP L={cfg['L']} h={cfg['h']}",
            "global_batch": B,
            "entries_per_sample": plan.entries_per_sample,
            "eloc_ms": eloc_ms,
            "chunk_samples": plan.chunk_samples,
            "energy": energy[0].item(),
        },
        "roofline": {
            "kernel": f"fused_forward<{prec},{cfg['h']}>",
            "bound": "mfma",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": None,
            "issued_tflops": executed,
            "ms_per_launch": fwd_ms_launch,
            "rows": prof["forward_rows"],
        },
    }

    if not args.no_fp32:
        P = min(args.fp32_prefix, B)
        plan32 = nqs.Plan(ctx, H, cfg["L"], cfg["h"], cfg["n_up"], cfg["n_dn"], "fp32", max_batch=P,
                          dedup=cfg["dedup"])
        xp = x[:P].contiguous()
        el32 = nqs.local_energy(plan32, params, xp)
        torch.cuda.synchronize()
        plan32.profile(True)
        el32 = nqs.local_energy(plan32, params, xp)
        p32 = plan32.profile_read()
        plan32.profile(False)
        v32 = P * K / (p32["eloc_ms"] / 1e3)
        wp = weights[:P]
        e_bf = np.sum(wp * eloc[:P, 0].cpu().numpy()) / np.sum(wp)
        e_32 = np.sum(wp * el32[:, 0].cpu().numpy()) / np.sum(wp)
        out["fp32_path"] = {"value": v32, "unit": "samples*terms/s", "prefix_samples": P,
                            "speedup_bf16_over_fp32": value / v32,
                            "energy_prefix_bf16_minus_fp32": float(e_bf - e_32),
                            "forward_tflops": p32["forward_flops"] / (p32["forward_ms"] / 1e3) / 1e12}
        log(f"fp32 path: {v32:.3e} samples*terms/s on {P} samples; bf16/fp32 = {value / v32:.2f}; "
            f"dE(prefix) = {e_bf - e_32:.3e}")
        del plan32

    if not args.no_cpu:
        from threadpoolctl import threadpool_info
        from oracle import made, pauli, vmc
        m = min(args.cpu_samples, B)
        ref = pauli.canonical_terms(terms.x_mask, terms.z_mask, terms.coeff)
        net = made.Net(n=cfg["n"], n_layers=cfg["L"], width=cfg["h"], n_up=cfg["n_up"], n_dn=cfg["n_dn"])
        t = time.time()
        el_ref = vmc.local_energy(ref, net, params_np, samples[:m])
        dt = time.time() - t
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
        gpu_el = eloc[:m].cpu().numpy()
        d_el = np.abs(gpu_el[:, 0] + 1j * gpu_el[:, 1] - el_ref)
        out["cpu_baseline"] = {"value": m * K / dt, "unit": "samples*terms/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"FP64 oracle local energy of the first {m} samples of the same "
                                         f"workload ({dt:.1f} s)",
                               "max_abs_dE_loc_vs_gpu": float(np.max(d_el))}
        log(f"oracle: {m} samples in {dt:.1f}s on {threads} threads; max |dE_loc| GPU vs oracle = "
            f"{np.max(d_el):.3e}")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
