#!/usr/bin/env python3
"""Benchmark of the local-energy + VMC-gradient step on one MI355X.

One step = nqs_energy_grad on one batch: sample forward, enumeration and
matrix elements of every connected configuration, the MFMA forward on all of
them, the FP64 ratio-and-reduce, the weighted energy and the hand backward.
Prints one JSON line; diagnostics go to stderr.

Default workload: 60 qubits (30 spatial orbitals, 15 up + 15 down electrons),
Jordan-Wigner Hamiltonian of the seeded molecular-like integral generator
(1,189,663 merged Pauli strings), a batch of 65,536 unique configurations
drawn from |psi|^2 by the GPU unique-sample sampler (10^12 draws, counts as
weights; --samples sector uses uniform sector draws instead), a BF16 masked
network L = 4, h = 1024 (BF16-valued parameters).  The timed path multiplies BF16 weights with
activations carried as two BF16 terms (two BF16 MFMAs, FP32 accumulation),
with FP64 matrix elements, sums and energy; the value is its local-energy
throughput B*K/t.  The whole step is also replayed from a HIP graph.

Beside it, on the first --prefix samples of the same batch and the same
network: the timed path again, the split-BF16, plain BF16 and FP32 GPU paths
(throughput + energy) and the FP64 GPU path (the energy reference of the
prefix); the timed path with the paper's separate phase sub-model and with
the forward and a random sampling order; one Adam step (Sec. 6) on the
network's parameters; the matrix elements from structured per-group tables
against the term list (enumeration of the first chunk, local energy of the
prefix); the timed network kind and shape at 76 qubits (bit
strings of two words; a sparser synthetic molecule with the paper's term
count for that size, uniform sector samples); and the FP64 CPU
oracle on --cpu-samples samples (CPU baseline, and the per-sample check of
every GPU path).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

ARITH = {"bf16w": "BF16 network (BF16-valued weights x two-term BF16 activations, 2 BF16 MFMAs, FP32 accumulation)",
         "bf16x3": "split-BF16 network (FP32 weights and activations as two BF16 terms, 3 BF16 MFMAs)",
         "bf16": "plain BF16 network", "fp32": "FP32 network", "fp64": "FP64 network"}
PEAKS_TFLOPS = {"bf16": 2500.0, "bf16x3": 2500.0, "bf16w": 2500.0, "fp32": 157.3, "fp64": 78.6}
METRIC = "E_loc samples\u00b7terms/s + VMC step ms, BF16 vs FP32 GPU at |\u0394E|\u22641e-5 Ha"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("paper_2208_05637_amd/csrc/kernels_forward.hip", "paper_2208_05637_amd/csrc/nqs_internal.h"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, prec, waves):
    """HBM bytes per configuration of the connected-configuration forward from
    the committed counter summary of this workload, or None when there is none
    or it was taken on another kernel source or workgroup shape."""
    path = os.path.join(ROOT, "profiles", f"fused_forward_{workload}_{prec}_traffic.md")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("|"):
                k, v = line.split(":", 1)
                kv[k.strip().strip("-* `")] = v.strip().strip("` ")
    try:
        if kv.get("kernel_source_sha256") != kernel_source_hash():
            return None
        return float(kv[f"traffic_bytes_per_row_w{waves}"])
    except (KeyError, ValueError):
        return None


# Bit strings of two words: 76 qubits, the size of the paper's largest system
# (38 spatial orbitals, 19 + 19 electrons).  The integrals' two-electron part
# is cut below 2.5e-5, which leaves about as many Pauli strings as the
# paper's 76-qubit molecule (1,625,991).
WIDE_N_ORB, WIDE_CUTOFF = 38, 2.5e-5


def wide_76(nqs, ctx, cfg, prec, count):
    """Local-energy throughput of the timed network kind and shape at 76 qubits,
    on `count` unique configurations drawn from the network by the GPU sampler
    (10^12 draws), workgroup shape and dedup autotuned."""
    import numpy as np
    import torch
    from gen.inputs import hamiltonian, init_params
    t = time.time()
    terms = hamiltonian(WIDE_N_ORB, 0, cutoff=WIDE_CUTOFF)
    log(f"76-qubit Hamiltonian: {len(terms)} strings in {time.time() - t:.1f}s")
    n, nu = 2 * WIDE_N_ORB, WIDE_N_ORB // 2
    H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
    params = torch.from_numpy(init_params(n, cfg["L"], cfg["h"], seed=1, dtype=cfg["params"])).to(ctx.device)
    pl = nqs.Plan(ctx, H, cfg["L"], cfg["h"], nu, nu, prec, max_batch=count, dedup="auto")
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record(ctx.stream)
    xs, _ = nqs.sample(pl, params, 10**12, seed=2, max_unique=count)
    s1.record(ctx.stream)
    torch.cuda.synchronize()
    count = xs.shape[0]
    pl.autotune(params, xs)               # workgroup shape and dedup, as for the main batch
    # connected configurations per distinct one over the batch (one chunk)
    con = nqs.connected(pl if pl.dedup else nqs.Plan(ctx, H, cfg["L"], cfg["h"], nu, nu, prec, max_batch=count,
                                                     dedup=True), xs)
    torch.cuda.synchronize()
    ratio = int(con["n_entries"].item()) / max(int(con["n_unique"].item()), 1)
    entries = int(con["n_entries"].item())
    del con
    nqs.local_energy(pl, params, xs)      # warm
    torch.cuda.synchronize()
    pl.profile(True)
    el = nqs.local_energy(pl, params, xs)
    pr = pl.profile_read()
    pl.profile(False)
    status = nqs.device_status(pl)
    el = el.cpu().numpy()
    res = {"n_qubits": n, "terms": H.K, "groups": H.G, "samples": count,
           "samples_kind": "unique configurations drawn from the network (10^12 draws)",
           "sampler_ms": s0.elapsed_time(s1),
           "entries_per_sample_bound": pl.entries_per_sample, "entries": entries, "dedup_ratio": ratio,
           "chunk_samples": pl.chunk_samples, "dedup": pl.dedup, "forward_rows": pr["forward_rows"],
           "forward_waves_per_block": pl.kernel_info()["waves_per_block"],
           "samples_terms_per_s": count * H.K / (pr["eloc_ms"] / 1e3),
           "connected_configs_per_s": pr["forward_rows"] / (pr["eloc_ms"] / 1e3),
           "forward_tflops": pr["forward_flops"] / (pr["forward_ms"] / 1e3) / 1e12,
           "forward_ms_per_launch": pr["forward_ms"] / max(pr["forward_launches"], 1),
           "energy_mean": float(np.mean(el[:, 0])), "device_status": status}
    log(f"76 qubits ({H.K} strings, {count} samples, {entries} entries, dedup ratio {ratio:.3f}, dedup "
        f"{'on' if pl.dedup else 'off'}): {res['samples_terms_per_s']:.3e} samples*terms/s, "
        f"{res['forward_tflops']:.1f} TFLOP/s")
    return res


def tables_side(nqs, ctx, terms, cfg, prec, waves, dedup, x, chunk, xp, params, ref):
    """Matrix elements from the structured tables (NQS_H_TABLES) against the term
    list: the enumeration of the batch's first chunk (diagonal, count, scan,
    write; no dedup), and the local energy of the prefix with the tables in
    the prefix path's configuration (ref: that path's result)."""
    import numpy as np
    import torch
    res = {}
    for tables in (False, True):
        Hh = nqs.Hamiltonian.from_terms(terms, tables=tables).upload(ctx)
        ep = nqs.Plan(ctx, Hh, cfg["L"], cfg["h"], cfg["n_up"], cfg["n_dn"], prec, max_batch=chunk,
                      chunk_samples=chunk)
        con = nqs.connected(ep, x[:chunk])      # warm
        del con
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        con = nqs.connected(ep, x[:chunk])
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        key = "tables" if tables else "term_list"
        res[f"enumeration_ms_first_chunk_{key}"] = e0.elapsed_time(e1)
        res[f"device_bytes_{key}"] = Hh.bytes
        res["entries_first_chunk"] = int(con["n_entries"].item())
        del con, ep
        if tables:
            P = xp.shape[0]
            pl = nqs.Plan(ctx, Hh, cfg["L"], cfg["h"], cfg["n_up"], cfg["n_dn"], prec, max_batch=P, dedup=dedup)
            pl.configure(waves_per_block=waves)
            nqs.local_energy(pl, params, xp)    # warm
            torch.cuda.synchronize()
            pl.profile(True)
            el = nqs.local_energy(pl, params, xp)
            pr = pl.profile_read()
            pl.profile(False)
            el = el.cpu().numpy()
            res["samples_terms_per_s_prefix"] = P * Hh.K / (pr["eloc_ms"] / 1e3)
            res["samples_terms_per_s_prefix_term_list"] = ref["value"]
            res["dedup"] = bool(dedup)
            res["max_abs_dE_loc_vs_term_list"] = float(np.max(np.abs(el - ref["eloc"])))
            del pl
        del Hh
    log(f"structured tables: first-chunk enumeration {res['enumeration_ms_first_chunk_tables']:.2f} ms "
        f"(term list {res['enumeration_ms_first_chunk_term_list']:.2f} ms); prefix "
        f"{res['samples_terms_per_s_prefix']:.3e} samples*terms/s (term list "
        f"{res['samples_terms_per_s_prefix_term_list']:.3e}); max |dE_loc| vs term list "
        f"{res['max_abs_dE_loc_vs_term_list']:.2e}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4", help="c1..c4, c5a..c5d")
    ap.add_argument("--batch", type=int, default=None, help="override the batch (diagnostic runs)")
    ap.add_argument("--precision", default=None, help="override the timed path's arithmetic")
    ap.add_argument("--prefix", type=int, default=1024, help="samples for the side paths")
    ap.add_argument("--cpu-samples", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-side", action="store_true", help="skip the prefix paths")
    ap.add_argument("--wide-samples", type=int, default=512,
                    help="samples of the 76-qubit side workload (0 skips it)")
    ap.add_argument("--chunk", type=int, default=0, help="samples per chunk (0 = plan default)")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (plan defaults)")
    ap.add_argument("--dedup", default=None, choices=["on", "off", "auto"],
                    help="override the workload's dedup setting")
    ap.add_argument("--waves", type=int, default=0, help="force the forward's waves per workgroup")
    ap.add_argument("--samples", default="psi", choices=["psi", "sector"],
                    help="psi: the batch is drawn from the network with the GPU unique-sample sampler "
                         "(1e12 draws, the batch size as buffer capacity); sector: uniform sector draws")
    ap.add_argument("--graph-steps", type=int, default=1,
                    help="replays of the HIP-graph-captured step after the timed steps (0 = none)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 3 device-to-device copies of MIB MiB (scale for HBM byte counters)")
    args = ap.parse_args()

    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.calibrate_copy, "copies": 3}))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the benchmark evaluates one GPU's share of the batch on a single MI355X; "
              "runs on several GPUs are not supported (the path would shard by samples, with one "
              "all-reduce of the gradient sums per step).", file=sys.stderr)
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
    log(f"inputs: n={cfg['n']} K terms generated, {time.time() - t:.1f}s")
    ctx = nqs.Context(0)
    H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
    K = H.K
    dev = ctx.device
    params = torch.from_numpy(params_np).to(dev)
    if args.dedup is not None:
        cfg["dedup"] = {"on": True, "off": False, "auto": "auto"}[args.dedup]
    mk = lambda p, mb: nqs.Plan(ctx, H, cfg["L"], cfg["h"], cfg["n_up"], cfg["n_dn"], p, max_batch=mb,
                                dedup=cfg["dedup"], chunk_samples=args.chunk)
    sampling = None
    if args.samples == "psi":
        # the batch: unique configurations drawn from |psi|^2 with their counts (Sec. 4, Sampling)
        want = cfg["B"] if args.batch is None else int(args.batch)
        splan = mk(prec, 16)
        nqs.sample(splan, params, 10**6, seed=1, max_unique=min(want, 1024))    # warm
        torch.cuda.synchronize()
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record(ctx.stream)
        xs_t, ws_t = nqs.sample(splan, params, 10**12, seed=2, max_unique=want)
        s1.record(ctx.stream)
        torch.cuda.synchronize()
        samples = xs_t.cpu().numpy().view(np.uint64).copy()
        weights = ws_t.cpu().numpy().copy()
        sampling = {"draws": 10**12, "unique": len(samples), "ms": s0.elapsed_time(s1), "seed": 2}
        log(f"sampler: {len(samples)} unique of 1e12 draws in {sampling['ms']:.1f} ms")
        del splan
    B = len(samples)
    plan = mk(prec, B)
    log(f"K={K} G={H.G} entries/sample={plan.entries_per_sample} chunk={plan.chunk_samples} "
        f"dedup={plan.dedup} workspace={plan.workspace_size(B) / 2**30:.2f} GiB")
    x = torch.from_numpy(samples.view(np.int64)).to(dev)
    w = torch.from_numpy(weights).to(dev)
    eloc = torch.empty((B, 2), dtype=torch.float64, device=dev)
    energy = torch.empty(3, dtype=torch.float64, device=dev)
    grad = torch.empty(plan.n_params, dtype=torch.float64, device=dev)
    plan.workspace(B)
    tune = None
    if args.waves:
        plan.configure(waves_per_block=args.waves)
    elif not args.no_tune:
        t = time.time()
        tune = plan.autotune(params, x)
        log(f"autotune ({time.time() - t:.1f}s, probe {tune['probe_samples']} samples): "
            + ", ".join(f"{c['waves_per_block']}w/dedup{int(c['dedup'])}/S{c['chunk_samples']}: {c['ms']:.1f} ms"
                        for c in tune["candidates"]) + f" -> {plan.kernel_info()}")

    for i in range(args.warmup):
        t = time.time()
        nqs.energy_grad(plan, params, x, w, eloc=eloc, energy=energy, grad=grad)
        torch.cuda.synchronize()
        log(f"warmup step {i}: {time.time() - t:.2f}s")

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
    if nqs.device_status(plan):
        raise RuntimeError("device error flag set during the timed steps")
    ms_step = ev0.elapsed_time(ev1) / args.steps
    eloc_ms = prof["eloc_ms"] / max(prof["calls"], 1)
    value = B * K / (eloc_ms / 1e3)
    log(f"step {ms_step:.1f} ms, local energy {eloc_ms:.1f} ms, E = {energy[0].item():.10f}")
    fwd_ms_launch = prof["forward_ms"] / max(prof["forward_launches"], 1)
    achieved = prof["forward_flops"] / (prof["forward_ms"] / 1e3) / 1e12
    issued = prof["forward_flops_executed"] / (prof["forward_ms"] / 1e3) / 1e12
    peak = PEAKS_TFLOPS[prec]
    log(f"forward kernel: {prof['forward_launches']} launches, {fwd_ms_launch:.2f} ms/launch, "
        f"{achieved:.1f} TFLOP/s algorithmic, {issued:.1f} TFLOP/s MFMA issued (peak {peak})")

    el_main = eloc.cpu().numpy()
    graph = None
    if args.graph_steps > 0:
        # the whole step (local energies, energy, gradient) as one captured HIP graph
        ref = (energy.clone(), grad.clone(), eloc.clone())
        gs = torch.cuda.Stream()
        ctx.use_stream(gs)
        try:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=gs):
                nqs.energy_grad(plan, params, x, w, eloc=eloc, energy=energy, grad=grad)
        finally:
            ctx.use_stream(torch.cuda.current_stream())
        energy.zero_(); grad.zero_(); eloc.zero_()
        torch.cuda.synchronize()
        # replay() launches on the current stream
        cur = torch.cuda.current_stream()
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        g0.record(cur)
        for i in range(args.graph_steps):
            g.replay()
        g1.record(cur)
        torch.cuda.synchronize()
        same = bool(torch.equal(energy, ref[0]) and torch.equal(grad, ref[1]) and torch.equal(eloc, ref[2]))
        graph = {"ms_per_step": g0.elapsed_time(g1) / args.graph_steps, "replays": args.graph_steps,
                 "equal_to_eager": same}
        log(f"graph-captured step: {graph['ms_per_step']:.1f} ms, equal to eager: {same}")
        del g
    # duplicates among the connected configurations: entries / distinct configurations of the
    # first chunk (what dedup would save; the autotuner decides whether the timed path uses it)
    dedup_ratio = None
    if not args.no_side and cfg["n"] < 64:
        dp = nqs.Plan(ctx, H, cfg["L"], cfg["h"], cfg["n_up"], cfg["n_dn"], prec, max_batch=plan.chunk_samples,
                      dedup=True, chunk_samples=plan.chunk_samples)
        con = nqs.connected(dp, x[:plan.chunk_samples])
        ne, nu = int(con["n_entries"].item()), int(con["n_unique"].item())
        dedup_ratio = ne / max(nu, 1)
        log(f"first chunk: {ne} connected configurations, {nu} distinct (ratio {dedup_ratio:.4f})")
        del con, dp
    adam = None
    if not args.no_side:
        # one Adam step (Sec. 6) on this network's parameters with the step's gradient, timed on its own
        pa = params.clone()
        opt = nqs.Adam(ctx, pa, lr=1e-3, betas=(0.9, 0.99))
        opt.step(grad)
        torch.cuda.synchronize()
        a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        a0.record(ctx.stream)
        for i in range(reps):
            opt.step(grad)
        a1.record(ctx.stream)
        torch.cuda.synchronize()
        ams = a0.elapsed_time(a1) / reps
        nb = 48 * pa.numel()       # p f32, g, m, v f64 read; p, m, v written
        adam = {"ms": ams, "params": pa.numel(), "alg_bytes": nb, "GB/s": nb / (ams / 1e3) / 1e9,
                "frac_of_hbm_peak": nb / (ams / 1e3) / 8e12}
        log(f"adam step: {ams * 1e3:.1f} us for {pa.numel()} parameters, {adam['GB/s']:.0f} GB/s")
        del opt, pa
    kinfo = plan.kernel_info()
    bpr = measured_traffic(args.workload, prec, kinfo["waves_per_block"])
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "samples*terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16w": "bf16", "bf16x3": "bf16x3", "bf16": "bf16", "fp32": "fp32", "fp64": "f64"}[prec],
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {cfg['n']} qubits ({cfg['N']} orbitals, {cfg['n_up']}+{cfg['n_dn']} "
                        f"electrons), K={K} Pauli strings, G={H.G} flips, B={B} unique samples "
                        f"(count weights, {'drawn from the network' if sampling else 'uniform in the sector'}), masked MLP L={cfg['L']} h={cfg['h']} with {cfg['params'].upper()} "
                        f"parameters, {ARITH[prec]}; FP64 matrix elements, sums and energy",
            "global_batch": B,
            "entries_per_sample": plan.entries_per_sample,
            "eloc_ms": eloc_ms,
            "chunk_samples": plan.chunk_samples,
            "dedup": plan.dedup,
            "forward_waves_per_block": kinfo["waves_per_block"],
            "forward_rows_per_block": kinfo["rows_per_block"],
            "autotuned": kinfo["tuned"],
            "energy": energy[0].item(),
            # every configuration of the spin sector has the same number of connected configurations
            # besides itself (the plan's per-sample entry bound is exact for these Hamiltonians)
            "connected_configs_per_s": B * plan.entries_per_sample / (eloc_ms / 1e3),
            "dedup_ratio": dedup_ratio,
        },
        "roofline": {
            "kernel": f"fused_forward<{prec},{cfg['h']}>",
            "bound": "mfma",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            # HBM bytes per launch: the counters' bytes per configuration times this run's
            # configurations per launch
            "traffic": (None if bpr is None else bpr * prof["forward_rows"] / max(prof["forward_launches"], 1)),
            "traffic_bytes_per_row": bpr,
            "alg_bytes_per_row": 24,
            "mfma_issued_tflops": issued,
            "mfma_issued_frac": issued / peak,
            # a multiply-add of two-term BF16 activations takes two BF16 MFMA products
            "products_per_mac": {"bf16w": 2, "bf16x3": 3}.get(prec, 1),
            "frac_of_product_peak": achieved * {"bf16w": 2, "bf16x3": 3}.get(prec, 1) / peak,
            "ms_per_launch": fwd_ms_launch,
            "rows": prof["forward_rows"],
            "alg_flop_per_row": prof["forward_flops"] / max(prof["forward_rows"], 1),
        },
    }

    out["config"]["samples"] = ("drawn from |psi|^2 by the GPU unique-sample sampler" if sampling
                                else "uniform over the spin sector, merged into counts")
    if sampling is not None:
        out["sampler"] = sampling
    if tune is not None:
        out["autotune"] = {"probe_samples": tune["probe_samples"], "from_cache": tune["from_cache"],
                           "candidates": tune["candidates"], "chosen": tune["chosen"]}
    if graph is not None:
        out["graph_step"] = graph
    if adam is not None:
        out["adam_step"] = adam

    side = {}
    P = min(args.prefix, B)
    if not args.no_side:
        xp = x[:P].contiguous()
        wp = weights[:P]
        for p in (prec, "bf16x3", "bf16", "fp32", "fp64"):
            if p in side:
                continue
            pl = mk(p, P)
            if p == prec:
                pl.configure(waves_per_block=kinfo["waves_per_block"])
            elif not args.no_tune and p != "fp64":
                pl.autotune(params, xp)
            nqs.local_energy(pl, params, xp)      # warm
            torch.cuda.synchronize()
            pl.profile(True)
            el = nqs.local_energy(pl, params, xp)
            pr = pl.profile_read()
            pl.profile(False)
            side[p] = dict(eloc=el.cpu().numpy(), value=P * K / (pr["eloc_ms"] / 1e3),
                           tflops=pr["forward_flops"] / (pr["forward_ms"] / 1e3) / 1e12)
            log(f"{p} path on {P} samples: {side[p]['value']:.3e} samples*terms/s, "
                f"{side[p]['tflops']:.1f} TFLOP/s")
            del pl
        Ep = {p: math.fsum(wp * d["eloc"][:, 0]) / math.fsum(wp) for p, d in side.items()}
        ref = Ep.get("fp64")
        acc = {}
        for p, d in side.items():
            acc[p] = {"samples_terms_per_s": d["value"], "forward_tflops": d["tflops"],
                      "energy_prefix": Ep[p],
                      "abs_dE_vs_fp64_gpu": None if ref is None else abs(Ep[p] - ref)}
        out["paths_on_prefix"] = {"prefix_samples": P, **acc}
        if "fp32" in side:
            # same samples, same network, each path with its own tuned kernel
            out["speedup_vs_fp32_path"] = side[prec]["value"] / side["fp32"]["value"]
        if ref is not None:
            out["abs_dE_prefix_vs_fp64"] = abs(Ep[prec] - ref)
        log("prefix energies: " + ", ".join(f"{p}={Ep[p]:.10f}" for p in Ep))

        # network variants on the same prefix, timed precision and workgroup shape: the paper's
        # separate phase sub-model, and the forward and a random sampling order
        from gen import init_params
        var = {}
        vspecs = [("separate_phase_network", dict(phase_mode=1)),
                  ("forward_order", dict(order=np.arange(cfg["n"]))),
                  ("random_order", dict(order=np.random.default_rng(5).permutation(cfg["n"])))]
        for name, kw in vspecs:
            vp = params
            if "phase_mode" in kw:
                vp = torch.from_numpy(init_params(cfg["n"], cfg["L"], cfg["h"], seed=1, dtype=cfg["params"],
                                                  phase_mode=1)).to(dev)
            pl = nqs.Plan(ctx, H, cfg["L"], cfg["h"], cfg["n_up"], cfg["n_dn"], prec, max_batch=P,
                          dedup=plan.dedup, chunk_samples=min(plan.chunk_samples, P), **kw)
            pl.configure(waves_per_block=kinfo["waves_per_block"])
            nqs.local_energy(pl, vp, xp)      # warm
            torch.cuda.synchronize()
            pl.profile(True)
            el = nqs.local_energy(pl, vp, xp)
            pr = pl.profile_read()
            pl.profile(False)
            ev = math.fsum(wp * el[:, 0].cpu().numpy()) / math.fsum(wp)
            var[name] = {"samples_terms_per_s": P * K / (pr["eloc_ms"] / 1e3),
                         "forward_tflops": pr["forward_flops"] / (pr["forward_ms"] / 1e3) / 1e12,
                         "alg_flop_per_row": pr["forward_flops"] / max(pr["forward_rows"], 1),
                         "energy_prefix": ev}
            log(f"variant {name}: {var[name]['samples_terms_per_s']:.3e} samples*terms/s, "
                f"{var[name]['forward_tflops']:.1f} TFLOP/s, E = {ev:.8f}")
            del pl
        out["variants_on_prefix"] = {"prefix_samples": P, "precision": prec, **var}

        if args.wide_samples > 0:
            out["wide_76_qubits"] = wide_76(nqs, ctx, cfg, prec, args.wide_samples)

        out["structured_tables"] = tables_side(nqs, ctx, terms, cfg, prec, kinfo["waves_per_block"], plan.dedup,
                                               x, plan.chunk_samples, xp, params, side[prec])

    if not args.no_cpu:
        from threadpoolctl import threadpool_info
        from oracle import made, pauli, vmc
        m = min(args.cpu_samples, B, P)
        refH = pauli.canonical_terms(terms.x_mask, terms.z_mask, terms.coeff)
        net = made.Net(n=cfg["n"], n_layers=cfg["L"], width=cfg["h"], n_up=cfg["n_up"], n_dn=cfg["n_dn"])
        t = time.time()
        el_ref = vmc.local_energy(refH, net, params_np, samples[:m])
        dt = time.time() - t
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
        checks = {}
        for p, d in ({**side, prec: dict(eloc=el_main)}).items():
            e = d["eloc"][:m]
            checks[p] = float(np.max(np.abs(e[:, 0] + 1j * e[:, 1] - el_ref)))
        out["cpu_baseline"] = {"value": m * K / dt, "unit": "samples*terms/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"FP64 oracle local energy of the first {m} samples of the "
                                         f"same workload ({dt:.1f} s)",
                               "max_abs_dE_loc_vs_oracle": checks}
        log(f"oracle: {m} samples in {dt:.1f}s on {threads} threads; max |dE_loc| vs oracle: {checks}")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
