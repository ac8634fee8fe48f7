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
network L = 4, h = 1024 (BF16-valued parameters).  The timed path multiplies
BF16 weights with activations carried as two BF16 terms (two BF16 MFMAs, FP32
accumulation), with FP64 matrix elements, sums and energy; the value is its
local-energy throughput B*K/t.

The run keeps to a wall-clock budget (--budget seconds from process start):
after the first warm-up step it times as many of the requested steps as fit
beside what still has to run, and reports the counts it ran.  Then: the step
replayed from a HIP graph (when it fits), one Adam step, and on the first
--prefix samples of the same batch and network the timed path, the FP32 GPU
path (the comparator of the speed-up) and the FP64 GPU path (the energy
reference of the prefix); then the FP64 CPU oracle on a time-bounded sample
(multi-threaded, and one sample on one thread).  Opt-in side workloads:
--all-paths (split and plain BF16 on the prefix), --variants (separate phase
sub-model, forward and random sampling orders), --wide-samples N (76 qubits,
two-word strings), --tables (structured matrix elements), --multi (the
four-instance workload in one call).  Workgroup shape, dedup and chunk come
from the committed tuner database when it holds the plan's key (--tune times
the candidates instead, --save-tune-db writes the choices).
"""
import time

T_START = time.time()   # the budget counts from here, before torch is imported

import argparse
import json
import math
import os
import sys

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
    for f in ("paper_2208_05637_amd/csrc/kernels_forward.hip", "paper_2208_05637_amd/csrc/net.h"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, prec, waves, rows):
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
        if kv.get("kernel_source_sha256") != kernel_source_hash() or kv.get("rows_per_block") != str(rows):
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


def tables_side(nqs, ctx, terms, cfg, prec, shape, dedup, x, chunk, xp, params, ref):
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
            pl.configure(waves_per_block=shape[0], rows_per_block=shape[1])
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


def multi_instances(nqs, ctx):
    """The four-instance workload in one nqs_energy_grad_multi call: 16, 28, 44
    and 64 qubits (seeds 1-4), each with its own Hamiltonian, BF16 network
    (L = 3, h = 512) and batch of 4,096 / 16,384 / 32,768 / 16,384 unique
    configurations drawn from that network by the GPU sampler."""
    import numpy as np
    import torch
    from gen import config_inputs
    dev = ctx.device
    items, keep, rows = [], [], []
    t = time.time()
    for name in ("c5a", "c5b", "c5c", "c5d"):
        terms, params_np, _, _, cfg = config_inputs(name, batch=16)
        H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
        p = torch.from_numpy(params_np).to(dev)
        sp = nqs.Plan(ctx, H, cfg["L"], cfg["h"], cfg["n_up"], cfg["n_dn"], cfg["precision"], max_batch=16)
        x, w = nqs.sample(sp, p, 10**12, seed=2, max_unique=cfg["B"])
        B = x.shape[0]
        plan = nqs.Plan(ctx, H, cfg["L"], cfg["h"], cfg["n_up"], cfg["n_dn"], cfg["precision"], max_batch=B,
                        dedup=cfg["dedup"])
        items.append(dict(plan=plan, params=p, samples=x, weights=w,
                          eloc=torch.empty((B, 2), dtype=torch.float64, device=dev),
                          energy=torch.empty(3, dtype=torch.float64, device=dev),
                          grad=torch.empty(plan.n_params, dtype=torch.float64, device=dev)))
        keep.append(H)
        rows.append(dict(n_qubits=cfg["n"], terms=H.K, samples=B, dedup=plan.dedup,
                         entries_per_sample=plan.entries_per_sample))
    log(f"four instances prepared in {time.time() - t:.1f}s")
    ws = nqs.multi_workspace(items)
    nqs.energy_grad_multi(items, ws)          # warm
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(ctx.stream)
    nqs.energy_grad_multi(items, ws)
    e1.record(ctx.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    status = nqs.multi_device_status(items, ws)
    for r, it in zip(rows, items):
        r["energy"] = float(it["energy"][0].item())
    st = sum(r["samples"] * r["terms"] for r in rows)
    res = {"ms_per_call": ms, "samples_terms_per_s": st / (ms / 1e3), "instances": rows, "device_status": status,
           "samples_kind": "unique configurations drawn from each instance's network (10^12 draws)"}
    log(f"four instances, one call: {ms:.1f} ms, {res['samples_terms_per_s']:.3e} samples*terms/s")
    return res


def cpu_baseline(terms, cfg, params_np, samples, seconds, gpu_paths):
    """The FP64 oracle on the host: local energies of the batch's first samples,
    one at a time until `seconds` have passed (BLAS on every thread it has),
    then the next sample on one thread.  The Hamiltonian's canonical form is
    built before the clock starts, as the GPU path's upload is."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import made, pauli, vmc
    refH = pauli.canonical_terms(terms.x_mask, terms.z_mask, terms.coeff)
    net = made.Net(n=cfg["n"], n_layers=cfg["L"], width=cfg["h"], n_up=cfg["n_up"], n_dn=cfg["n_dn"])
    els = []
    t0 = time.time()
    while len(els) < len(samples) - 1 and (not els or time.time() - t0 < seconds):
        els.append(vmc.local_energy(refH, net, params_np, samples[len(els):len(els) + 1])[0])
    dt = time.time() - t0
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    m = len(els)
    with threadpool_limits(1):
        t1 = time.time()
        els.append(vmc.local_energy(refH, net, params_np, samples[m:m + 1])[0])
        dt1 = time.time() - t1
    el_ref = np.array(els)
    checks = {}
    for p, e in gpu_paths.items():
        e = e[:m + 1]
        checks[p] = float(np.max(np.abs(e[:, 0] + 1j * e[:, 1] - el_ref)))
    return {"m": m, "dt": dt, "threads": threads, "dt1": dt1, "checks": checks}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--budget", type=float, default=440.0,
                    help="wall-clock seconds from process start the run keeps to (timed steps are cut to fit)")
    ap.add_argument("--workload", default="c4", help="c1..c4, c5a..c5d")
    ap.add_argument("--batch", type=int, default=None, help="override the batch (diagnostic runs)")
    ap.add_argument("--precision", default=None, help="override the timed path's arithmetic")
    ap.add_argument("--prefix", type=int, default=1024, help="samples for the prefix paths")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="seconds of multi-threaded oracle work (at least one sample), then one sample on "
                         "one thread")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-side", action="store_true", help="skip the prefix paths, graph replay and Adam step")
    ap.add_argument("--all-paths", action="store_true", help="also split and plain BF16 on the prefix")
    ap.add_argument("--variants", action="store_true", help="network variants on the prefix")
    ap.add_argument("--wide-samples", type=int, default=0,
                    help="samples of the 76-qubit side workload (0 skips it)")
    ap.add_argument("--tables", action="store_true", help="structured matrix elements side line")
    ap.add_argument("--multi", action="store_true", help="four-instance workload side line")
    ap.add_argument("--chunk", type=int, default=0, help="samples per chunk (0 = plan default)")
    ap.add_argument("--tune", action="store_true", help="time the tuner's candidates (not from the database)")
    ap.add_argument("--tune-db", default=os.path.join(ROOT, "paper_2208_05637_amd", "tune_db.txt"))
    ap.add_argument("--save-tune-db", default=None, metavar="PATH", help="write the tuner's choices here")
    ap.add_argument("--dedup", default=None, choices=["on", "off", "auto"],
                    help="override the workload's dedup setting")
    ap.add_argument("--waves", type=int, default=0, help="force the forward's waves per workgroup")
    ap.add_argument("--resident", type=int, default=None, choices=[0, 1],
                    help="with --waves: force the forward's grid (1 resident workgroups, 0 one per tile)")
    ap.add_argument("--samples", default="psi", choices=["psi", "sector"],
                    help="psi: the batch is drawn from the network with the GPU unique-sample sampler "
                         "(1e12 draws, the batch size as buffer capacity); sector: uniform sector draws")
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

    if args.tune:
        os.environ.setdefault("NQS_TUNE_LOG", "1")   # the tuner reports each candidate as it is timed
    import numpy as np
    import torch
    import paper_2208_05637_amd as nqs
    from gen import config_inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    elapsed = lambda: time.time() - T_START
    log(f"torch and the package imported at {elapsed():.1f}s")

    db_entries = 0
    if args.tune_db and os.path.exists(args.tune_db):
        db_entries = nqs.tune_db_load(args.tune_db)

    t = time.time()
    terms, params_np, samples, weights, cfg = config_inputs(args.workload, batch=args.batch)
    prec = args.precision or cfg["precision"]
    log(f"inputs: n={cfg['n']}, {len(terms.coeff)} strings generated in {time.time() - t:.1f}s")
    ctx = nqs.Context(0)
    H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
    K = H.K
    dev = ctx.device
    params = torch.from_numpy(params_np).to(dev)
    if args.dedup is not None:
        cfg["dedup"] = {"on": True, "off": False, "auto": "auto"}[args.dedup]
    mk = lambda p, mb: nqs.Plan(ctx, H, cfg["L"], cfg["h"], cfg["n_up"], cfg["n_dn"], p, max_batch=mb,
                                dedup=cfg["dedup"], chunk_samples=args.chunk)

    def tuned(pl, xs):
        """Apply the database's choice for this plan (or time the candidates with --tune)."""
        if args.waves:
            pl.configure(waves_per_block=args.waves, resident=None if args.resident is None else bool(args.resident))
            return None
        if args.tune:
            return pl.autotune(params, xs, force=True)
        info = pl.autotune(params, xs[:1], cache_only=True)
        return info if info["from_cache"] else None

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
    x = torch.from_numpy(samples.view(np.int64)).to(dev)
    w = torch.from_numpy(weights).to(dev)
    eloc = torch.empty((B, 2), dtype=torch.float64, device=dev)
    energy = torch.empty(3, dtype=torch.float64, device=dev)
    grad = torch.empty(plan.n_params, dtype=torch.float64, device=dev)
    plan.workspace(B)
    if args.tune:
        # the tuner times its probe, which needs warm kernels
        plan.autotune(params, x[:64], force=True)
    tune = tuned(plan, x)
    kinfo = plan.kernel_info()
    log(f"K={K} G={H.G} entries/sample={plan.entries_per_sample} chunk={plan.chunk_samples} "
        f"dedup={plan.dedup} waves={kinfo['waves_per_block']} rows={kinfo['rows_per_block']} "
        f"resident={kinfo['resident']} tuned={kinfo['tuned']} "
        f"workspace={plan.workspace_size(B) / 2**30:.2f} GiB")
    if tune is not None and not tune["from_cache"]:
        log("autotune: " + ", ".join(f"{c['waves_per_block']}w/{c['rows_per_block']}r/dedup{int(c['dedup'])}/"
                                    f"S{c['chunk_samples']}/"
                                    f"{'resident' if c['resident'] else 'tiles'}: {c['ms']:.1f} ms"
                                    for c in tune["candidates"]))

    # first warm-up step, which also prices one step for the budget
    t = time.time()
    nqs.energy_grad(plan, params, x, w, eloc=eloc, energy=energy, grad=grad)
    torch.cuda.synchronize()
    T_step = time.time() - t
    warm_run = 1
    log(f"warmup step 0: {T_step:.2f}s (at {elapsed():.1f}s)")
    # what still runs after the timed steps: prefix paths, graph replay (one step), the CPU oracle
    reserve = (0.0 if args.no_side else 20.0 + T_step) + (0.0 if args.no_cpu else 2.5 * args.cpu_seconds + 10.0)
    fit = int((args.budget - elapsed() - reserve) // max(T_step, 1e-3))
    steps = max(1, min(args.steps, fit))
    extra_warm = max(0, min(args.warmup - 1, fit - steps))
    if steps < args.steps:
        log(f"budget {args.budget:.0f}s: {steps} of {args.steps} timed steps fit")
    for i in range(extra_warm):
        nqs.energy_grad(plan, params, x, w, eloc=eloc, energy=energy, grad=grad)
        torch.cuda.synchronize()
        warm_run += 1
        log(f"warmup step {warm_run - 1} done at {elapsed():.1f}s")

    plan.profile(True)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(ctx.stream)
    for i in range(steps):
        nqs.energy_grad(plan, params, x, w, eloc=eloc, energy=energy, grad=grad)
        if T_step > 2.0:
            # a progress line per long step (the wait between steps costs microseconds of a step)
            torch.cuda.synchronize()
            log(f"timed step {i} done at {elapsed():.1f}s")
    ev1.record(ctx.stream)
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    if nqs.device_status(plan):
        raise RuntimeError("device error flag set during the timed steps")
    ms_step = ev0.elapsed_time(ev1) / steps
    eloc_ms = prof["eloc_ms"] / max(prof["calls"], 1)
    value = B * K / (eloc_ms / 1e3)
    log(f"{steps} timed steps: {ms_step:.1f} ms per step, local energy {eloc_ms:.1f} ms, "
        f"E = {energy[0].item():.10f} (at {elapsed():.1f}s)")
    fwd_ms_launch = prof["forward_ms"] / max(prof["forward_launches"], 1)
    achieved = prof["forward_flops"] / (prof["forward_ms"] / 1e3) / 1e12
    issued = prof["forward_flops_executed"] / (prof["forward_ms"] / 1e3) / 1e12
    peak = PEAKS_TFLOPS[prec]
    log(f"forward kernel: {prof['forward_launches']} launches, {fwd_ms_launch:.2f} ms/launch, "
        f"{achieved:.1f} TFLOP/s algorithmic, {issued:.1f} TFLOP/s MFMA issued (peak {peak})")
    el_main = eloc.cpu().numpy()
    E_main = energy.cpu().numpy()
    bpr = measured_traffic(args.workload, prec, kinfo["waves_per_block"], kinfo["rows_per_block"])
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "samples*terms/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm_run,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16w": "bf16", "bf16x3": "bf16x3", "bf16": "bf16", "fp32": "fp32", "fp64": "f64"}[prec],
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {cfg['n']} qubits ({cfg['N']} orbitals, {cfg['n_up']}+{cfg['n_dn']} "
                        f"electrons), K={K} Pauli strings, G={H.G} flips, B={B} unique samples "
                        f"(count weights, {'drawn from the network' if sampling else 'uniform in the sector'}), "
                        f"masked MLP L={cfg['L']} h={cfg['h']} with {cfg['params'].upper()} "
                        f"parameters, {ARITH[prec]}; FP64 matrix elements, sums and energy",
            "global_batch": B,
            "steps_requested": args.steps,
            "warmup_requested": args.warmup,
            "budget_s": args.budget,
            "entries_per_sample": plan.entries_per_sample,
            "eloc_ms": eloc_ms,
            "chunk_samples": plan.chunk_samples,
            "dedup": plan.dedup,
            "forward_waves_per_block": kinfo["waves_per_block"],
            "forward_rows_per_block": kinfo["rows_per_block"],
            "forward_resident_grid": kinfo["resident"],
            "tuned": kinfo["tuned"],
            "tune_from_db": bool(tune is not None and tune["from_cache"] and not args.tune),
            "energy": float(E_main[0]),
            # every configuration of the spin sector has the same number of connected configurations
            # besides itself (the plan's per-sample entry bound is exact for these Hamiltonians)
            "connected_configs_per_s": B * plan.entries_per_sample / (eloc_ms / 1e3),
            "forward_rows_per_step": prof["forward_rows"] / steps,
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
            "ms_per_launch": fwd_ms_launch,
            "launches": prof["forward_launches"],
            "rows": prof["forward_rows"],
            "alg_flop_per_row": prof["forward_flops"] / max(prof["forward_rows"], 1),
        },
    }
    out["config"]["samples"] = ("drawn from |psi|^2 by the GPU unique-sample sampler" if sampling
                                else "uniform over the spin sector, merged into counts")
    if sampling is not None:
        out["sampler"] = sampling
    if tune is not None:
        out["autotune"] = {"from_db": bool(tune["from_cache"]) and not args.tune,
                           "probe_samples": tune["probe_samples"],
                           "candidates": tune["candidates"], "chosen": tune["chosen"]}

    side = {}
    P = min(args.prefix, B)
    gpu_paths = {prec: el_main}
    if not args.no_side:
        # the same step replayed from one captured HIP graph (local energies, energy, gradient)
        if args.budget - elapsed() - (2.5 * args.cpu_seconds + 30.0) >= T_step:
            gs = torch.cuda.Stream()
            ctx.use_stream(gs)
            try:
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=gs):
                    nqs.energy_grad(plan, params, x, w, eloc=eloc, energy=energy, grad=grad)
            finally:
                ctx.use_stream(torch.cuda.current_stream())
            energy.zero_(); grad.zero_(); eloc.zero_()
            ref_grad = None
            torch.cuda.synchronize()
            cur = torch.cuda.current_stream()
            g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            g0.record(cur)
            g.replay()
            g1.record(cur)
            torch.cuda.synchronize()
            same = bool(np.array_equal(energy.cpu().numpy(), E_main) and np.array_equal(eloc.cpu().numpy(), el_main))
            out["graph_step"] = {"ms_per_step": g0.elapsed_time(g1), "replays": 1, "equal_to_eager": same}
            log(f"graph-captured step: {g0.elapsed_time(g1):.1f} ms, equal to eager: {same}")
            del g
        else:
            out["graph_step"] = {"skipped": "time budget"}
        # one Adam step (Sec. 6) on this network's parameters with the step's gradient
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
        out["adam_step"] = {"ms": ams, "params": pa.numel(), "alg_bytes": nb, "GB/s": nb / (ams / 1e3) / 1e9,
                            "frac_of_hbm_peak": nb / (ams / 1e3) / 8e12}
        del opt, pa

        # the prefix paths: same samples, same network, each path in its tuned configuration
        xp = x[:P].contiguous()
        wp = weights[:P]
        paths = [prec, "fp32", "fp64"] + (["bf16x3", "bf16"] if args.all_paths else [])
        for p in dict.fromkeys(paths):
            pl = mk(p, P)
            if p != "fp64":                                  # (the FP64 reference runs untuned)
                if args.tune:
                    pl.autotune(params, xp[:64], force=True)     # warm kernels for the tuner's timing
                tuned(pl, xp)
            nqs.local_energy(pl, params, xp[:64])            # warm
            torch.cuda.synchronize()
            pl.profile(True)
            el = nqs.local_energy(pl, params, xp)
            pr = pl.profile_read()
            pl.profile(False)
            side[p] = dict(eloc=el.cpu().numpy(), value=P * K / (pr["eloc_ms"] / 1e3),
                           tflops=pr["forward_flops"] / (pr["forward_ms"] / 1e3) / 1e12,
                           waves=pl.kernel_info()["waves_per_block"])
            log(f"{p} path on {P} samples: {side[p]['value']:.3e} samples*terms/s, "
                f"{side[p]['tflops']:.1f} TFLOP/s")
            del pl
        Ep = {p: math.fsum(wp * d["eloc"][:, 0]) / math.fsum(wp) for p, d in side.items()}
        ref = Ep["fp64"]
        out["paths_on_prefix"] = {"prefix_samples": P, **{
            p: {"samples_terms_per_s": d["value"], "forward_tflops": d["tflops"], "waves_per_block": d["waves"],
                "energy_prefix": Ep[p], "abs_dE_vs_fp64_gpu": abs(Ep[p] - ref)} for p, d in side.items()}}
        out["speedup_vs_fp32_path"] = side[prec]["value"] / side["fp32"]["value"]
        out["abs_dE_prefix_vs_fp64"] = abs(Ep[prec] - ref)
        log("prefix energies: " + ", ".join(f"{p}={Ep[p]:.10f}" for p in Ep))
        for p, d in side.items():
            if p != prec:
                gpu_paths[p] = d["eloc"]

    if not args.no_cpu:
        t = time.time()
        cb = cpu_baseline(terms, cfg, params_np, samples, args.cpu_seconds, gpu_paths)
        m = cb["m"]
        out["cpu_baseline"] = {
            "value": m * K / cb["dt"], "unit": "samples*terms/s", "cores": cb["threads"], "kind": "oracle",
            "sample": f"FP64 oracle local energies of the first {m} samples of the same batch, one sample "
                      f"at a time ({cb['dt']:.1f} s on {cb['threads']} BLAS threads); sample {m + 1} on one "
                      f"thread ({cb['dt1']:.1f} s)",
            "single_thread": {"value": K / cb["dt1"], "unit": "samples*terms/s", "cores": 1,
                              "samples": 1, "seconds": cb["dt1"]},
            "max_abs_dE_loc_vs_oracle": cb["checks"]}
        log(f"oracle: {m} samples in {cb['dt']:.1f}s on {cb['threads']} threads, 1 sample in {cb['dt1']:.1f}s on "
            f"one thread; max |dE_loc| vs oracle: {cb['checks']} (at {elapsed():.1f}s)")

    # opt-in side workloads (each guarded: the headline line is printed whatever they do)
    def guarded(name, fn):
        try:
            out[name] = fn()
        except Exception as e:        # a side line never costs the headline
            log(f"{name} failed: {e!r}")
            out[name] = {"error": repr(e)}

    if args.variants:
        def variants():
            from gen import init_params
            xp = x[:P].contiguous()
            wp = weights[:P]
            var = {}
            for name, kw in [("separate_phase_network", dict(phase_mode=1)),
                             ("forward_order", dict(order=np.arange(cfg["n"]))),
                             ("random_order", dict(order=np.random.default_rng(5).permutation(cfg["n"])))]:
                vp = params
                if "phase_mode" in kw:
                    vp = torch.from_numpy(init_params(cfg["n"], cfg["L"], cfg["h"], seed=1, dtype=cfg["params"],
                                                      phase_mode=1)).to(dev)
                pl = nqs.Plan(ctx, H, cfg["L"], cfg["h"], cfg["n_up"], cfg["n_dn"], prec, max_batch=P,
                              dedup=plan.dedup, chunk_samples=min(plan.chunk_samples, P), **kw)
                pl.configure(waves_per_block=kinfo["waves_per_block"], rows_per_block=kinfo["rows_per_block"],
                             resident=kinfo["resident"])
                nqs.local_energy(pl, vp, xp[:64])
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
                log(f"variant {name}: {var[name]['samples_terms_per_s']:.3e} samples*terms/s")
                del pl
            return {"prefix_samples": P, "precision": prec, **var}
        guarded("variants_on_prefix", variants)
    if args.wide_samples > 0:
        guarded("wide_76_qubits", lambda: wide_76(nqs, ctx, cfg, prec, args.wide_samples))
    if args.tables and "paths_on_prefix" in out:
        guarded("structured_tables", lambda: tables_side(
            nqs, ctx, terms, cfg, prec, (kinfo["waves_per_block"], kinfo["rows_per_block"]), plan.dedup, x,
            plan.chunk_samples, x[:P].contiguous(), params, side[prec]))
    if args.multi:
        guarded("multi_instance", lambda: multi_instances(nqs, ctx))
    if args.save_tune_db:
        nqs.tune_db_save(args.save_tune_db)
        log(f"tuner database written to {args.save_tune_db}")
    out["wall_s"] = elapsed()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
