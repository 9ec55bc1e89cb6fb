#!/usr/bin/env python3
"""Throughput of the MCMC surface-code decoder on one MI355X.

Workload (the metric point): distance L = 13 planar code, depolarizing
p = 0.15, 4 classes x 4 chains, 169 = L^2 counted sweeps, single temperature
(beta* = beta_bar), decided per syndrome.  A step decodes one batch of
syndromes that is already resident in device memory: class starts, the
colour-phased Metropolis chains, the estimator and the decision, all in the
library's kernels.  Batches are sampled on the device before timing (distinct
sample ids per step) with the library's depolarizing sampler.

Printed: one JSON line with syndromes/s (value), stabilizer updates/s, the
logical error rate of the decoded batches, the integer-ALU roofline of the
chain kernel (its duration measured with events on the launch stream as the
difference between a full step and a step with no sweeps) and the CPU oracle
timed on a bounded sample of the same workload.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

L, P, CHAINS, SWEEPS, BURN, K = 13, 0.15, 4, 169, 0, 1
Q_BITPHASE = 0.10
SEED = 0x1302266900000013
BATCH = 65536
# integer operations per stabilizer update in the minimal scalar formulation:
# Philox4x32-10 share 20 (5 mul_lo + 5 mul_hi + 10 xor), weight change 8-12,
# accept 4, flip 4, accumulate 3 -> 40 at the low end
OPS_PER_UPDATE = 40
# random scan: two uniforms per step (40), the site pick (a high multiply, 1),
# weight change, accept and flip as above (16) and the per-step sums (3)
RS_OPS_PER_UPDATE = 60
# MI355X vector ALU: 256 CUs x 128 lanes per clock x 2.4 GHz = 78.6 T lane
# slots/s (the FP32 vector peak of 157.3 TFLOP/s counts an FMA as two flops);
# three-operand integer instructions (v_mad_u64_u32: mul_lo + mul_hi,
# v_bitop3: two XORs, v_add3: two adds) retire two operations per slot, so the
# integer-operation peak is 157.3 T ops/s
PEAK_INT_OPS = 256 * 128 * 2.4e9 * 2
# HBM traffic of the chain kernel from rocprofv3 FETCH_SIZE (x2.000, the
# counter's reading of a 256 MiB copy) + WRITE_SIZE (x1.000) at 65536 syndromes
# per launch (the counters file under profiles/ for chains_r0 at L=13): bytes
# per syndrome, valid only for the kernel sources it was measured on
CHAIN_TRAFFIC_PER_SYNDROME = 81232846 / 65536
# (file, first line, line after) of the sources the chain kernel is built from:
# whole files, and internal.h from the launch descriptors to the kernel-range
# table (the rest of that header declares other kernels)
CHAIN_TRAFFIC_SOURCES = (("chain_body.h", None, None), ("chain_r0.hip", None, None),
                         ("device_common.h", None, None),
                         ("internal.h", "struct GroupDesc {", "hipError_t launch_chains("))
CHAIN_TRAFFIC_SHA = "0940c00ba5a05ddf"
# gate network at L=13: 2 flops per multiply-add over the three 3x3 convolutions
# (3->32, 32->32, 32->32 on 169 pixels) and the 5408x7 head
CNN_FLOPS_PER_SAMPLE = 2 * (169 * 32 * 27 + 2 * 169 * 32 * 288 + 7 * 5408)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=BATCH)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=256)
    ap.add_argument("--no-budget-curve", action="store_true",
                    help="skip the logical error vs sweep budget curve")
    ap.add_argument("--workload", choices=["metric", "mixed", "gated", "bitphase", "spacetime",
                                           "randomscan", "context"],
                    default="metric",
                    help="metric: L=13 p=0.15 (default); mixed: L in 5..25, p in [0.05,0.18]; "
                         "gated: gate network trained and timed against the plain decoder; "
                         "bitphase: L=13, independent bit/phase flips q=0.10; "
                         "spacetime: L=7, 7 measurement rounds, p = p_M = 0.02")
    ap.add_argument("--gate-train", type=int, default=1_000_000)
    ap.add_argument("--gate-epochs", type=int, default=4)
    ap.add_argument("--gate-eval", type=int, default=100_000)
    ap.add_argument("--gap-max-miss", type=float, default=0.003,
                    help="gated workload: bound on the fraction of gap-routed training "
                         "samples whose decision needs sweeps, per rate bin")
    ap.add_argument("--mixed-n", type=int, default=100000)
    ap.add_argument("--st-L", type=int, default=0,
                    help="space-time workload: code distance (default 7)")
    ap.add_argument("--st-rounds", type=int, default=0,
                    help="space-time workload: measurement rounds (default = L)")
    ap.add_argument("--st-sweeps", type=int, default=0,
                    help="space-time workload: sweeps (default 16 L^2)")
    ap.add_argument("--init", choices=["greedy", "mwpm"], default="mwpm",
                    help="class starts: Sec. III's exact enhanced matching (default), or the "
                         "greedy matching")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run one device copy of this size (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the decoder "
              "shards by syndrome with no exchange, so a multi-GPU figure is not produced.",
              file=sys.stderr)
        sys.exit(2)

    # the oracle baseline first, in forked workers, before anything touches the GPU
    args.cpu = None
    if not args.no_cpu_baseline and args.workload in ("metric", "bitphase", "randomscan",
                                                      "spacetime"):
        ns = 2 * L * (L - 1)
        if args.workload == "metric":
            args.cpu = cpu_baseline(args.cpu_sample, ns, workers=host_cores(),
                                    init=args.init)
        elif args.workload == "bitphase":
            args.cpu = cpu_baseline(args.cpu_sample, ns, noise=1, p=Q_BITPHASE,
                                    workers=host_cores())
        elif args.workload == "randomscan":
            args.cpu = cpu_baseline(min(args.cpu_sample, 64), ns, random_scan=True,
                                    workers=host_cores())
        elif not args.st_L:   # the oracle baseline is for the default space-time workload
            args.cpu = cpu_baseline_spacetime(host_cores())

    import torch
    import paper_1302_2669_amd as mc
    args.init_mode = mc.MCMC_INIT_MWPM if args.init == "mwpm" else mc.MCMC_INIT_MATCHING

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "mixed":
        return bench_mixed(args, mc, torch, dev)
    if args.workload == "gated":
        return bench_gated(args, mc, torch, dev)
    if args.workload == "bitphase":
        return bench_bitphase(args, mc, torch, dev)
    if args.workload == "spacetime":
        return bench_spacetime(args, mc, torch, dev)
    if args.workload == "randomscan":
        return bench_randomscan(args, mc, torch, dev)
    if args.workload == "context":
        return bench_context(args, mc, torch, dev)
    n = args.batch
    nq, ns = mc.geometry(L)
    steps, warm = args.steps, args.warmup

    # resident inputs: one distinct batch per step
    batches, truth = [], []
    for b in range(warm + steps):
        syn, cls, _ = mc.sample_errors(L, P, SEED, n, device=dev, id_base=b * n)
        batches.append(syn)
        truth.append(cls)
    prm = mc.make_params(L, P, SWEEPS, SEED, chains=CHAINS, n_temps=K, burn=BURN)
    ws = torch.empty((mc.workspace_size(prm, n),), dtype=torch.uint8, device=dev)
    ids = [torch.arange(b * n, (b + 1) * n, dtype=torch.int32, device=dev)
           for b in range(warm + steps)]
    torch.cuda.synchronize()

    def step(b, sweeps=SWEEPS, burn=BURN, workspace=ws):
        return mc.decode_batch(batches[b], L, P, sweeps, SEED, chains=CHAINS, n_temps=K,
                               burn=burn, syndrome_ids=ids[b], want_correction=True,
                               workspace=workspace, init=args.init_mode)

    for b in range(warm):
        step(b)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    chosen = []
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        out = step(warm + i)
        ev[i + 1].record(stream)
        chosen.append(out["chosen"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    ms_per_step = wall * 1e3 / steps

    # same launches with no sweep: class starts + estimator only
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(steps):
        step(warm + i, sweeps=0)
    e1.record(stream)
    torch.cuda.synchronize()
    overhead_ms = e0.elapsed_time(e1) / steps
    chain_ms = float(np.mean(per_step_ms)) - overhead_ms

    updates_per_syndrome = 4 * CHAINS * K * (BURN + SWEEPS) * ns
    syn_per_s = n * steps / wall
    upd_per_s = syn_per_s * updates_per_syndrome
    fails = sum(int((c != t).sum().item()) for c, t in zip(chosen, truth[warm:]))
    total = n * steps
    p_l = fails / total
    z = 1.96
    den = 1 + z * z / total
    centre = (p_l + z * z / (2 * total)) / den
    half = z * np.sqrt(p_l * (1 - p_l) / total + z * z / (4 * total * total)) / den

    chain_updates = n * updates_per_syndrome
    achieved = chain_updates * OPS_PER_UPDATE / (chain_ms * 1e-3) / 1e12
    peak = PEAK_INT_OPS / 1e12

    # logical error vs sweep budget on the same syndromes and chains (chains
    # are keyed by sweep, so a shorter budget is a prefix of the same run):
    # the smallest budget within 2% relative of the full one is the
    # matched-error operating point
    curve = None
    if not args.no_budget_curve:
        nb = min(4, steps)
        full_chosen = chosen[:nb]
        curve = []
        # counted sweeps (burn-in 0) from L^2/8 to 4 L^2, and L^2 split into
        # L^2/2 uncounted + L^2/2 counted (same cost as L^2)
        points = [(0, 0), (SWEEPS // 8, 0), (SWEEPS // 4, 0), (SWEEPS // 2, 0), (SWEEPS, 0),
                  (2 * SWEEPS, 0), (4 * SWEEPS, 0), (SWEEPS - SWEEPS // 2, SWEEPS // 2)]
        ws_big = None
        for b, burn in points:
            if b + burn > SWEEPS and ws_big is None:
                ws_big = torch.empty((mc.workspace_size(mc.make_params(
                    L, P, 4 * SWEEPS, SEED, chains=CHAINS, n_temps=K), n),),
                    dtype=torch.uint8, device=dev)
            outs = []
            c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            c0.record(stream)
            for i in range(nb):
                outs.append(step(warm + i, sweeps=b, burn=burn,
                                 workspace=ws if ws_big is None else ws_big)["chosen"])
            c1.record(stream)
            torch.cuda.synchronize()
            ms_b = c0.elapsed_time(c1) / nb
            wrong = sum(int((o != t).sum().item()) for o, t in zip(outs, truth[warm:warm + nb]))
            right_full = [f == t for f, t in zip(full_chosen, truth[warm:warm + nb])]
            right_b = [o == t for o, t in zip(outs, truth[warm:warm + nb])]
            worse = sum(int((rf & ~rb).sum().item()) for rf, rb in zip(right_full, right_b))
            better = sum(int((~rf & rb).sum().item()) for rf, rb in zip(right_full, right_b))
            curve.append({"sweeps": b, "burn": burn, "logical_error": wrong / (n * nb),
                          "syndromes_per_s": n / (ms_b * 1e-3),
                          "full_right_budget_wrong": worse, "full_wrong_budget_right": better})
        ref_err = next(c for c in curve if c["sweeps"] == SWEEPS and c["burn"] == 0)["logical_error"]
        for c in curve:
            c["rel_error_change"] = (c["logical_error"] - ref_err) / ref_err
        matched = next(c for c in curve if c["rel_error_change"] <= 0.02)

    # the same batches from the other start (greedy matching, or the exact
    # matching when the greedy one is timed), for comparison
    other = mc.MCMC_INIT_MATCHING if args.init == "mwpm" else mc.MCMC_INIT_MWPM
    no = min(4, steps)
    o0, o1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    o0.record(stream)
    other_chosen = [mc.decode_batch(batches[warm + i], L, P, SWEEPS, SEED, chains=CHAINS,
                                    n_temps=K, burn=BURN, syndrome_ids=ids[warm + i],
                                    want_correction=True, workspace=ws, init=other)["chosen"]
                    for i in range(no)]
    o1.record(stream)
    torch.cuda.synchronize()
    other_wrong = sum(int((c != t).sum().item()) for c, t in zip(other_chosen, truth[warm:]))
    other_start = {"start": "greedy" if args.init == "mwpm" else "mwpm",
                   "syndromes_per_s": n * no / (o0.elapsed_time(o1) * 1e-3),
                   "logical_error": other_wrong / (n * no), "samples": n * no}

    # end to end: syndromes from pinned host memory, decisions, class
    # probabilities and corrections back to pinned host memory, same stream
    ne = min(4, steps)
    h_syn = [batches[warm + i].cpu().pin_memory() for i in range(ne)]
    h_chosen = torch.empty((n,), dtype=torch.uint8).pin_memory()
    h_prob = torch.empty((n, 4), dtype=torch.float64).pin_memory()
    h_corr = torch.empty((n, nq), dtype=torch.uint8).pin_memory()
    d_syn = torch.empty_like(batches[0])
    torch.cuda.synchronize()
    t_e2e = time.perf_counter()
    for i in range(ne):
        d_syn.copy_(h_syn[i], non_blocking=True)
        o = mc.decode_batch(d_syn, L, P, SWEEPS, SEED, chains=CHAINS, n_temps=K, burn=BURN,
                            syndrome_ids=ids[warm + i], want_correction=True, workspace=ws,
                            init=args.init_mode)
        h_chosen.copy_(o["chosen"], non_blocking=True)
        h_prob.copy_(o["class_prob"], non_blocking=True)
        h_corr.copy_(o["correction"], non_blocking=True)
        torch.cuda.synchronize()
        if i == 0 and not torch.equal(h_chosen, chosen[0].cpu()):
            raise RuntimeError("end-to-end decisions differ from the resident run")
    e2e = {"syndromes_per_s": n * ne / (time.perf_counter() - t_e2e), "steps": ne,
           "note": "syndromes copied in from pinned host memory and decisions, class "
                   "probabilities and corrections copied back, on the decode stream, "
                   "synchronised per batch"}

    copy_probe(args, torch, dev)

    cpu = args.cpu

    line = {
        "metric": "decoded syndromes/sec + stabilizer updates/sec at L=13 p=0.15, matched logical error",
        "value": syn_per_s,
        "unit": "syndromes/s",
        "stabilizer_updates_per_s": upd_per_s,
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic: i.i.d. depolarizing samples from the library's Philox sampler",
        "config": {"workload": "planar code L=13, depolarizing p=0.15, 4 classes x 4 chains, "
                               "169 sweeps (L^2), single temperature, batch of "
                               f"{n} syndromes per step, "
                               + ("exact enhanced-matching starts (Sec. III)" if args.init == "mwpm"
                                  else "greedy matching starts"),
                   "start": args.init,
                   "L": L, "p": P, "chains_per_class": CHAINS, "sweeps": SWEEPS, "burn": BURN,
                   "n_temps": K, "batch": n, "updates_per_syndrome": updates_per_syndrome},
        "logical_error": {"rate": p_l, "wilson95": [centre - half, centre + half],
                          "samples": total},
        "roofline": {"bound": "alu", "kernel": "chains_r0_kernel (L 2..13, at L=13)",
                     "achieved": achieved, "peak": peak, "unit": "Tops/s",
                     "frac": achieved / peak, "traffic": chain_traffic(n),
                     "traffic_unit": "bytes per launch",
                     "algorithmic_bytes": n * (4 * 104 + 16 * 20 + 4 * 100),
                     "chain_ms_per_launch": chain_ms, "ops_per_update": OPS_PER_UPDATE,
                     "updates_per_launch": chain_updates},
        "cpu_baseline": cpu,
        "end_to_end": e2e,
        "starts_and_estimator_ms_per_step": overhead_ms,
        "other_start": other_start,
        "budget_curve": curve,
        "matched_error_budget": None if curve is None else
            {"sweeps": matched["sweeps"], "syndromes_per_s": matched["syndromes_per_s"],
             "rel_error_change": matched["rel_error_change"],
             "note": "smallest counted budget (no burn-in) within 2% relative of the L^2 "
                     "logical error on the same syndromes and chains"},
    }
    if curve is not None and other_start["start"] == "greedy":
        # the cheapest budget from the exact matching starts whose logical error
        # is at most that of the greedy starts at L^2 sweeps, same syndromes
        ok = [c for c in curve if c["burn"] == 0 and
              c["logical_error"] <= other_start["logical_error"]]
        if ok:
            best = min(ok, key=lambda c: c["sweeps"])
            line["vs_greedy_start_at_matched_error"] = {
                "sweeps": best["sweeps"], "logical_error": best["logical_error"],
                "syndromes_per_s": best["syndromes_per_s"],
                "greedy_L2_logical_error": other_start["logical_error"],
                "greedy_L2_syndromes_per_s": other_start["syndromes_per_s"],
                "speedup": best["syndromes_per_s"] / other_start["syndromes_per_s"]}
    print(json.dumps(line), flush=True)


def chain_traffic(n):
    """Measured HBM bytes of one chain-kernel launch of n syndromes, or None
    when the kernel sources differ from the ones the counters were taken on."""
    import hashlib
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1302_2669_amd", "csrc")
    h = hashlib.sha256()
    for f, first, after in CHAIN_TRAFFIC_SOURCES:
        with open(os.path.join(here, f), "r") as fh:
            text = fh.read()
        if first is not None:
            i = text.find(first)
            j = text.find(after, i)
            if i < 0 or j < 0:
                return None
            text = text[i:j]
        h.update(text.encode())
    if h.hexdigest()[:16] != CHAIN_TRAFFIC_SHA:
        return None
    return CHAIN_TRAFFIC_PER_SYNDROME * n


def copy_probe(args, torch, dev):
    """A plain device-to-device copy of --copy-probe-mb MiB, for scaling the
    HBM byte counters of a profiled run."""
    if args.copy_probe_mb:
        src = torch.ones((args.copy_probe_mb << 20,), dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()


def bench_mixed(args, mc, torch, dev):
    """Mixed sizes in one plan: L uniform in {5, 7, ..., 25}, p uniform in
    [0.05, 0.18], budget L^2 sweeps, 4 chains per class; autotuned launch
    shape, graph-captured execution."""
    from paper_1302_2669_amd.inputs import mixed_workload
    n = args.mixed_n
    Ls, ps, sweeps = mixed_workload(n, seed=SEED ^ 0x3)
    items = [dict(L=int(l), p=float(q), sweeps=int(s), chains=4, syndrome_id=i)
             for i, (l, q, s) in enumerate(zip(Ls, ps, sweeps))]
    plan = mc.MixedPlan(items, seed=SEED)
    syn, cls = plan.sample(SEED, device=dev)
    tuning = plan.autotune(syn)
    out = plan.execute(syn, graph=True)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        plan.execute(syn, graph=True, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    fail = float((out["chosen"] != cls).float().mean())
    line = {
        "metric": "decoded syndromes/sec, mixed L 5..25 in one plan",
        "value": n * args.steps / wall, "unit": "syndromes/s",
        "stabilizer_updates_per_s": plan.total_updates * args.steps / wall,
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic: i.i.d. depolarizing samples per item",
        "config": {"workload": f"{n} syndromes, L uniform in {{5,...,25}}, p uniform in "
                               "[0.05,0.18], L^2 sweeps, 4 chains per class, one plan",
                   "tuning": tuning, "updates_per_step": plan.total_updates},
        "logical_error": {"rate": fail, "samples": n},
        # the five range kernels together over the whole execution (starts and
        # estimator included, under 1% of it)
        "roofline": {"bound": "alu", "kernel": "chains_r0..r4_kernel (whole plan)",
                     "achieved": plan.total_updates * OPS_PER_UPDATE / (ms * 1e-3) / 1e12,
                     "peak": PEAK_INT_OPS / 1e12, "unit": "Tops/s",
                     "frac": plan.total_updates * OPS_PER_UPDATE / (ms * 1e-3) / PEAK_INT_OPS,
                     "traffic": None, "ms_per_execution": ms,
                     "ops_per_update": OPS_PER_UPDATE},
    }
    print(json.dumps(line), flush=True)


def bench_gated(args, mc, torch, dev):
    """The gate network at L=13: trained on the GPU on decoder-made labels for
    syndromes with p uniform in [0.05, 0.18], then the gated decoder and the
    plain decoder (every syndrome at L^2 sweeps, one graph-captured plan)
    decode the same fresh syndromes with the same chains.  Reported at the
    fastest setting whose logical error stays within 2% relative of the plain
    decoder's (the matched-error operating point), with the rest of the
    trade-off beside it."""
    from scipy.stats import binomtest
    from paper_1302_2669_amd import gate
    from paper_1302_2669_amd.inputs import uniform_rates
    seed = SEED ^ 0x5
    init = args.init_mode
    n_tr, n_ev = args.gate_train, args.gate_eval

    def now():
        torch.cuda.synchronize()
        return time.perf_counter()

    t0 = now()
    p_tr = uniform_rates(n_tr, seed).astype(np.float64)
    syn, _, ids = gate.sample_dataset(L, p_tr, seed, id_base=0)
    # class targets relative to the start decision: the class head then says
    # whether (and how) the no-sweep answer is wrong
    soft, bud, _ = gate.mcmc_labels(L, syn, p_tr, ids, seed, init=init, relative=True)
    start_right = float(soft[:, 0].mean())
    label_mix = [float((bud == k).float().mean()) for k in range(3)]
    # the start-weight gap route's thresholds, fitted on the same labels
    gap_table = gate.fit_gap_table(p_tr, mc.start_weights(syn, L, init=init), bud,
                                   args.gap_max_miss, 50)
    t1 = now()
    net = gate.GateNet(L, gate.init_params(L, seed, device=dev), device=dev)
    hist = gate.train(net, syn, torch.from_numpy(p_tr.astype(np.float32)).to(dev), soft, bud,
                      epochs=args.gate_epochs, batch=512, lr=3e-3, seed=seed)
    t2 = now()
    del syn, soft, bud

    def measure(p_ev, tag):
        syn_e, cls_e, ids_e = gate.sample_dataset(L, p_ev, seed + 7, id_base=1 << 30)
        # a perfect gate: the evaluation syndromes' own budget labels
        _, bud_e, _ = gate.mcmc_labels(L, syn_e, p_ev, ids_e, seed, label_temps=2, init=init)
        mix = [int((bud_e == k).sum()) for k in range(3)]
        bound = n_ev * SWEEPS / max(1, mix[1] * L + mix[2] * SWEEPS)
        plan = mc.MixedPlan.from_arrays(L, p_ev, SWEEPS, seed, chains=CHAINS, syndrome_ids=ids_e,
                                        init=init)
        flat = syn_e.reshape(-1)
        out = plan.execute(flat, want_correction=True, graph=True)
        reps = max(1, args.steps // 2)
        ta = now()
        for _ in range(reps):
            out = plan.execute(flat, want_correction=True, graph=True, out=out)
        t_plain = (now() - ta) / reps
        plan.close()
        pr = out["chosen"] == cls_e
        err_plain = float((~pr).float().mean())
        points = []
        # (threshold, escalation margin, class route, gap route); threshold 1
        # leaves the network no route 0 or 1: the gap route alone
        for thr, esc, cr, gp in ((0.99, 0.0, True, False), (0.99, 0.0, False, False),
                                 (0.99, 3.0, False, False), (0.95, 0.0, True, False),
                                 (0.95, 3.0, False, False), (0.9, 3.0, False, False),
                                 (0.9, 0.0, True, False), (1.0, 0.0, False, True),
                                 (0.995, 0.0, True, True), (0.99, 0.0, True, True),
                                 (0.99, 3.0, False, True), (0.95, 3.0, False, True)):
            g = gate.GatedDecoder(L, P, seed, max_batch=n_ev, chains=CHAINS, threshold=thr,
                                  escalate=esc, init=init, class_route=cr,
                                  gap_table=gap_table if gp else None)
            res = g.decode(net.params, syn_e, p=p_ev, ids=ids_e, want_correction=True)
            ta = now()
            for _ in range(reps):
                res = g.decode(net.params, syn_e, p=p_ev, ids=ids_e, want_correction=True)
            t_g = (now() - ta) / reps
            g.close()
            gr = res["chosen"] == cls_e
            c = res["counts"]
            work = c[1] * L + (c[2] + c[3]) * SWEEPS + c[3] * L
            err = float((~gr).float().mean())
            b_dis, c_dis = int((pr & ~gr).sum()), int((~pr & gr).sum())
            mcnemar = binomtest(b_dis, b_dis + c_dis, 0.5).pvalue if b_dis + c_dis else 1.0
            # syndromes the class head answered with a class other than the
            # start decision
            zc = res["logits"][:, :4]
            conf = torch.softmax(zc, dim=1).max(dim=1).values
            moved = int(((conf >= thr) & (zc.argmax(dim=1) != 0)).sum()) if cr else 0
            points.append({"threshold": thr, "escalate": esc, "class_route": cr,
                           "gap_route": gp,
                           "class_head_other_class": moved, "syndromes_per_s": n_ev / t_g,
                           "speedup": t_plain / t_g, "work_saving": n_ev * SWEEPS / max(1, work),
                           "logical_error": err, "rel_error_change": (err - err_plain) / err_plain,
                           "plain_right_gated_wrong": b_dis, "plain_wrong_gated_right": c_dis,
                           "mcnemar_p": mcnemar, "routes": c})
        # the network alone over the evaluation batch: the fused inference
        # kernel the gated decoder runs, and the layered training forward
        pe = torch.from_numpy(p_ev.astype(np.float32)).to(dev)
        stream = torch.cuda.current_stream(dev)

        def timed(fn):
            fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        _, ws_f = gate.forward(L, net.params, syn_e, pe)
        _, ws_i = gate.infer(L, net.params, syn_e, pe)
        fwd_ms = timed(lambda: gate.forward(L, net.params, syn_e, pe, ws_f))
        inf_ms = timed(lambda: gate.infer(L, net.params, syn_e, pe, ws_i))
        del ws_f
        return {"workload": tag, "plain_syndromes_per_s": n_ev / t_plain,
                "plain_logical_error": err_plain, "points": points,
                "perfect_gate": {"budget_mix": mix, "work_saving_bound": bound,
                                 "note": "fraction of syndromes whose plain decision is already "
                                         "final with no sweep / L sweeps (labels of the "
                                         "evaluation syndromes themselves)"},
                "cnn_infer_ms": inf_ms, "cnn_forward_layered_ms": fwd_ms}

    uni = measure(uniform_rates(n_ev, seed + 1).astype(np.float64),
                  "L=13, p uniform in [0.05,0.18]")
    fix = measure(np.full(n_ev, P), "L=13, p=0.15")
    # the matched-error operating point: the fastest decoder, the plain one
    # included (the gate is switched off when it does not pay), whose logical
    # error is within 2% relative of the plain decoder's on the same syndromes
    plain_point = {"threshold": None, "escalate": None, "class_route": None, "gap_route": None,
                   "gate": "off",
                   "syndromes_per_s": uni["plain_syndromes_per_s"], "speedup": 1.0,
                   "rel_error_change": 0.0}
    matched = [q for q in uni["points"] if q["rel_error_change"] <= 0.02] + [plain_point]
    head = max(matched, key=lambda q: q["syndromes_per_s"])
    flops_fwd = n_ev * CNN_FLOPS_PER_SAMPLE
    line = {
        "metric": "decoded syndromes/sec, gated decoder (trained gate network) vs plain MCMC",
        "value": head["syndromes_per_s"], "unit": "syndromes/s",
        "n_gpus": 1, "steps": max(1, args.steps // 2), "warmup": 1,
        "ms_per_step": 1e3 * n_ev / head["syndromes_per_s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16+u32",
        "data": "synthetic: i.i.d. depolarizing samples; labels from the decoder itself",
        "config": {"workload": f"L=13, p uniform in [0.05,0.18]: gate network trained on {n_tr} "
                               f"decoder-labelled syndromes ({args.gate_epochs} epochs), "
                               f"{n_ev} evaluation syndromes, budgets 0 / L / L^2, "
                               "4 classes x 4 chains",
                   "labels_s": t1 - t0, "train_s": t2 - t1, "final_train_loss": hist[-1],
                   "start": args.init, "train_budget_label_mix": label_mix,
                   "train_mean_p_start_decision_right": start_right,
                   "class_targets": "relative to the start decision",
                   "escalate": "replica margin z of the short run's decision",
                   "gap_table": {"max_miss": args.gap_max_miss, "min_count": 50,
                                 "thresholds_by_rate_bin": [int(v) for v in gap_table]}},
        "speedup_vs_plain": head["speedup"],
        "operating_point": {"threshold": head["threshold"], "escalate": head["escalate"],
                            "class_route": head["class_route"], "gap_route": head["gap_route"],
                            "gate": head.get("gate", "on"),
                            "rel_error_change": head["rel_error_change"],
                            "rule": "fastest decoder (plain included) within 2% relative "
                                    "logical error of plain"},
        "results": [uni, fix],
        "roofline": {"bound": "mfma", "kernel": "infer_kernel (fused gate network inference)",
                     "achieved": flops_fwd / (uni["cnn_infer_ms"] * 1e-3) / 1e12,
                     "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": flops_fwd / (uni["cnn_infer_ms"] * 1e-3) / 1e12 / 2500.0,
                     "traffic": None, "flops_per_sample": CNN_FLOPS_PER_SAMPLE,
                     "samples_per_launch": n_ev},
    }
    print(json.dumps(line), flush=True)


def bench_bitphase(args, mc, torch, dev):
    """Independent bit/phase flips (Eq. pauliChannel with p_b = p_p = q) at
    the rate the paper studies for this model, q = 0.10, L = 13, 4 x 4
    chains, L^2 sweeps at beta* = 0.85 beta_bar (the paper's choice for this
    model).  Also the logical error at beta*/beta_bar = 0.70, 0.85 and 1.00
    on the same syndromes and chains."""
    q, bp = Q_BITPHASE, mc.MCMC_NOISE_BITPHASE
    n, steps, warm = args.batch, args.steps, args.warmup
    nq, ns = mc.geometry(L)
    batches, truth = [], []
    for b in range(warm + steps):
        syn, cls, _ = mc.sample_errors(L, q, SEED, n, device=dev, id_base=b * n, noise=bp)
        batches.append(syn)
        truth.append(cls)
    prm = mc.make_params(L, q, SWEEPS, SEED, chains=CHAINS, noise=bp)
    ws = torch.empty((mc.workspace_size(prm, n),), dtype=torch.uint8, device=dev)
    ids = [torch.arange(b * n, (b + 1) * n, dtype=torch.int32, device=dev)
           for b in range(warm + steps)]
    torch.cuda.synchronize()

    def step(b, sweeps=SWEEPS, scale=0.0):
        return mc.decode_batch(batches[b], L, q, sweeps, SEED, chains=CHAINS, syndrome_ids=ids[b],
                               want_correction=True, workspace=ws, noise=bp, beta_scale=scale)

    for b in range(warm):
        step(b)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    chosen = []
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        chosen.append(step(warm + i)["chosen"])
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = float(np.mean([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(steps):
        step(warm + i, sweeps=0)
    e1.record(stream)
    torch.cuda.synchronize()
    chain_ms = step_ms - e0.elapsed_time(e1) / steps
    updates_per_syndrome = 4 * CHAINS * SWEEPS * ns
    achieved = n * updates_per_syndrome * OPS_PER_UPDATE / (chain_ms * 1e-3) / 1e12
    peak = PEAK_INT_OPS / 1e12
    fails = sum(int((c != t).sum().item()) for c, t in zip(chosen, truth[warm:]))
    total = n * steps
    nb = min(4, steps)
    scan = []
    for scale in (0.70, 0.85, 1.00):
        outs = [step(warm + i, scale=scale)["chosen"] for i in range(nb)]
        wrong = sum(int((o != t).sum().item()) for o, t in zip(outs, truth[warm:warm + nb]))
        scan.append({"beta_scale": scale, "logical_error": wrong / (n * nb), "samples": n * nb})
    cpu = args.cpu
    line = {
        "metric": "decoded syndromes/sec + stabilizer updates/sec at L=13, independent "
                  "bit/phase flips q=0.10",
        "value": total / wall,
        "unit": "syndromes/s",
        "stabilizer_updates_per_s": total / wall * updates_per_syndrome,
        "n_gpus": 1, "steps": steps, "warmup": warm, "ms_per_step": wall * 1e3 / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic: i.i.d. bit and phase flips from the library's Philox sampler",
        "config": {"workload": "planar code L=13, independent bit/phase flips q=0.10, 4 classes "
                               "x 4 chains, 169 sweeps (L^2), beta* = 0.85 beta_bar, batch of "
                               f"{n} syndromes per step",
                   "L": L, "q": q, "chains_per_class": CHAINS, "sweeps": SWEEPS, "batch": n,
                   "beta_scale": 0.85, "updates_per_syndrome": updates_per_syndrome},
        "logical_error": {"rate": fails / total, "samples": total},
        "beta_scale_scan": scan,
        "roofline": {"bound": "alu", "kernel": "chains_flip_r0_kernel (L 2..13, at L=13)",
                     "achieved": achieved, "peak": peak, "unit": "Tops/s",
                     "frac": achieved / peak, "traffic": None,
                     "chain_ms_per_launch": chain_ms, "ops_per_update": OPS_PER_UPDATE,
                     "updates_per_launch": n * updates_per_syndrome},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def bench_spacetime(args, mc, torch, dev):
    """Imperfect measurements (Sec. VI): L = 7, T = 7 rounds (the last one
    perfect), depolarizing p = 0.02 per interval and outcome error p_M = 0.02,
    4 classes x 4 chains, 784 = 16 L^2 sweeps of every spatial and time move
    (the local moves relax slowly in space-time), 32768 histories per step
    (524288 chains: 8192 one-wave workgroups, 8 waves on each of the 1024
    SIMDs, the register-resident kernel's full residency).
    Also the logical error of decoding the last round alone with the
    single-round decoder (L^2 sweeps), on the same histories."""
    Ls, T, p, pm, chains, sweeps = ST_L, ST_T, ST_P, ST_PM, ST_CHAINS, ST_SWEEPS
    if args.st_L:
        Ls = args.st_L
        T = args.st_rounds or Ls
        sweeps = args.st_sweeps or 16 * Ls * Ls
    n = 32768
    steps, warm = args.steps, args.warmup
    nq, ns = mc.geometry(Ls)
    hist, truth = [], []
    for b in range(warm + steps):
        o, c = mc.sample_spacetime(Ls, T, p, pm, SEED, n, device=dev, id_base=b * n)
        hist.append(o)
        truth.append(c)
    prm = mc.spacetime_params(Ls, T, p, pm, sweeps, SEED, chains)
    import ctypes
    from paper_1302_2669_amd import _lib
    b_ = ctypes.c_size_t()
    _lib.check(_lib._lib().mcmc_spacetime_workspace_size(ctypes.byref(prm), n, ctypes.byref(b_)),
               "mcmc_spacetime_workspace_size")
    ws = torch.empty((b_.value,), dtype=torch.uint8, device=dev)
    ids = [torch.arange(b * n, (b + 1) * n, dtype=torch.int32, device=dev)
           for b in range(warm + steps)]

    def step(b, sw=sweeps):
        return mc.decode_spacetime(hist[b], Ls, p, pm, sw, SEED, chains=chains,
                                   syndrome_ids=ids[b], want_correction=True, workspace=ws)

    for b in range(warm):
        step(b)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    chosen = []
    t0 = time.perf_counter()
    e0.record(stream)
    for i in range(steps):
        chosen.append(step(warm + i)["chosen"])
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = e0.elapsed_time(e1) / steps
    z0, z1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    z0.record(stream)
    for i in range(steps):
        step(warm + i, sw=0)
    z1.record(stream)
    torch.cuda.synchronize()
    chain_ms = step_ms - z0.elapsed_time(z1) / steps
    copy_probe(args, torch, dev)
    moves_per_history = 4 * chains * sweeps * (T * ns + 2 * (T - 1) * nq)
    achieved = n * moves_per_history * OPS_PER_UPDATE / (chain_ms * 1e-3) / 1e12
    fails = sum(int((c != t).sum().item()) for c, t in zip(chosen, truth[warm:]))
    total = n * steps
    p_eff = 1 - (1 - p) ** T
    last_fail = 0
    for i in range(steps):
        out = mc.decode_batch(hist[warm + i][:, T - 1].contiguous(), Ls, p_eff, Ls * Ls, SEED,
                              chains=chains, want_correction=False)
        last_fail += int((out["chosen"] != truth[warm + i]).sum().item())
    line = {
        "metric": f"decoded measurement histories/sec, imperfect measurements (L={Ls}, {T} rounds)",
        "value": total / wall, "unit": "histories/s",
        "moves_per_s": total / wall * moves_per_history,
        "n_gpus": 1, "steps": steps, "warmup": warm, "ms_per_step": wall * 1e3 / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32+f64",
        "data": "synthetic: depolarizing data errors and wrong outcomes from the library's "
                "Philox sampler",
        "config": {"workload": f"planar code L={Ls}, T={T} measurement rounds (last perfect), "
                               f"p = p_M = 0.02, 4 classes x 4 chains, {sweeps} sweeps of all "
                               f"spatial and time moves, {n} histories per step",
                   "L": Ls, "rounds": T, "p": p, "p_m": pm, "chains_per_class": chains,
                   "sweeps": sweeps, "batch": n, "moves_per_history": moves_per_history},
        "logical_error": {"rate": fails / total, "samples": total,
                          "last_round_only": last_fail / total},
        "roofline": {"bound": "alu",
                     "kernel": (f"st_chain_fast_kernel<{Ls}>" if Ls <= 12 else
                                f"st_chain_win_kernel<{Ls}>") + " (space-time chains)",
                     "achieved": achieved, "peak": PEAK_INT_OPS / 1e12, "unit": "Tops/s",
                     "frac": achieved / (PEAK_INT_OPS / 1e12), "traffic": None,
                     "chain_ms_per_launch": chain_ms, "ops_per_update": OPS_PER_UPDATE,
                     "updates_per_launch": n * moves_per_history},
        "cpu_baseline": args.cpu,
    }
    print(json.dumps(line), flush=True)


def bench_randomscan(args, mc, torch, dev):
    """The paper's own random-scan chain (Sec. IV: one stabilizer picked at
    random per step, n summed after every step) at the metric point: L = 13,
    p = 0.15, 4 x 4 chains, 169 sweeps of n_stab steps.  A cross-check of the
    colour-phased scan, not the throughput path."""
    n, steps, warm = args.batch, args.steps, args.warmup
    nq, ns = mc.geometry(L)
    batches, truth = [], []
    for b in range(warm + steps):
        syn, cls, _ = mc.sample_errors(L, P, SEED, n, device=dev, id_base=b * n)
        batches.append(syn)
        truth.append(cls)
    prm = mc.make_params(L, P, SWEEPS, SEED, chains=CHAINS, flags=mc.MCMC_RANDOM_SCAN)
    ws = torch.empty((mc.workspace_size(prm, n),), dtype=torch.uint8, device=dev)
    ids = [torch.arange(b * n, (b + 1) * n, dtype=torch.int32, device=dev)
           for b in range(warm + steps)]
    torch.cuda.synchronize()

    def step(b, sweeps=SWEEPS):
        return mc.decode_batch(batches[b], L, P, sweeps, SEED, chains=CHAINS, syndrome_ids=ids[b],
                               want_correction=True, workspace=ws, random_scan=True)

    for b in range(warm):
        step(b)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    chosen = []
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        chosen.append(step(warm + i)["chosen"])
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = float(np.mean([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(steps):
        step(warm + i, sweeps=0)
    e1.record(stream)
    torch.cuda.synchronize()
    chain_ms = step_ms - e0.elapsed_time(e1) / steps
    updates_per_syndrome = 4 * CHAINS * SWEEPS * ns
    achieved = n * updates_per_syndrome * RS_OPS_PER_UPDATE / (chain_ms * 1e-3) / 1e12
    peak = PEAK_INT_OPS / 1e12
    fails = sum(int((c != t).sum().item()) for c, t in zip(chosen, truth[warm:]))
    total = n * steps
    cpu = args.cpu
    line = {
        "metric": "decoded syndromes/sec + stabilizer updates/sec at L=13 p=0.15, random scan",
        "value": total / wall,
        "unit": "syndromes/s",
        "stabilizer_updates_per_s": total / wall * updates_per_syndrome,
        "n_gpus": 1, "steps": steps, "warmup": warm, "ms_per_step": wall * 1e3 / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic: i.i.d. depolarizing samples from the library's Philox sampler",
        "config": {"workload": "planar code L=13, depolarizing p=0.15, 4 classes x 4 chains, "
                               "169 sweeps of n_stab random-site steps, single temperature, "
                               f"batch of {n} syndromes per step",
                   "L": L, "p": P, "chains_per_class": CHAINS, "sweeps": SWEEPS, "batch": n,
                   "updates_per_syndrome": updates_per_syndrome},
        "logical_error": {"rate": fails / total, "samples": total},
        "roofline": {"bound": "alu", "kernel": "chains_random_kernel (at L=13)",
                     "achieved": achieved, "peak": peak, "unit": "Tops/s",
                     "frac": achieved / peak, "traffic": None,
                     "chain_ms_per_launch": chain_ms, "ops_per_update": RS_OPS_PER_UPDATE,
                     "updates_per_launch": n * updates_per_syndrome},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def bench_context(args, mc, torch, dev):
    """Logical error rates set beside the paper's own figures (context, not a
    throughput line).  (a) Sec. IV.A's proof-of-principle point: at
    depolarizing p = 0.13 the single-temperature decoder's logical error falls
    below p from L = 6 on.  (b) Its threshold of 15-16%: logical error against
    p for several L, where curves of growing L cross.  The paper starts its
    chains from enhanced matching and samples L^4 steps per chain (about L^2/2
    sweeps).  4 classes x 4 chains, class starts from --init, budgets of 0
    (the decision of the starts alone: with the exact enhanced-matching starts
    this is Sec. III's enhanced-matching decoder), L^2/2, L^2 and 4 L^2 sweeps
    (65536, 65536, 32768 and 16384 syndromes per point)."""
    z = 1.96

    def point(L, p, frac, n, seed):
        sweeps = int(round(frac * L * L))
        syn, cls, _ = mc.sample_errors(L, p, seed, n, device=dev)
        out = mc.decode_batch(syn, L, p, sweeps, seed, chains=CHAINS, want_correction=False,
                              init=args.init_mode)
        wrong = int((out["chosen"] != cls).sum().item())
        r = wrong / n
        den = 1 + z * z / n
        c = (r + z * z / (2 * n)) / den
        h = z * np.sqrt(r * (1 - r) / n + z * z / (4 * n * n)) / den
        return {"L": L, "p": p, "sweeps": sweeps, "logical_error": r,
                "wilson95": [c - h, c + h], "samples": n}

    t0 = time.perf_counter()
    small, scan = [], []
    for frac, n in ((0.0, args.batch), (0.5, args.batch), (1.0, args.batch // 2),
                    (4.0, args.batch // 4)):
        small += [point(L, 0.13, frac, n, SEED + 100 + L) for L in (4, 5, 6, 7, 8)]
        scan += [point(L, p, frac, n, SEED + 1000 * L + int(p * 1000))
                 for L in (9, 13, 17, 21, 25) for p in (0.14, 0.15, 0.16, 0.17)]
        print(f"context: budget {frac} L^2 done, {time.perf_counter() - t0:.0f} s",
              file=sys.stderr, flush=True)
    start = ("exact enhanced-matching starts (Sec. III)" if args.init == "mwpm"
             else "greedy matching starts")
    line = {
        "metric": "logical error rate beside the paper's figures (context)",
        "value": None, "unit": "logical error", "n_gpus": 1, "higher_is_better": False,
        "data": "synthetic: i.i.d. depolarizing samples from the library's Philox sampler",
        "config": {"workload": f"depolarizing noise, {start}, 4 classes x 4 chains, "
                               "0, L^2/2, L^2 and 4 L^2 sweeps", "start": args.init},
        "proof_of_principle_p013": small,
        "threshold_scan": scan,
        "seconds": time.perf_counter() - t0,
    }
    print(json.dumps(line), flush=True)


def _oracle_shard(job):
    """One worker's shard: decode syndromes with ids [lo, lo + n) on the
    oracle; returns the seconds it took."""
    lo, n, noise, p, random_scan, init = job
    here = os.path.dirname(os.path.abspath(__file__))
    if here not in sys.path:
        sys.path.insert(0, here)
    from oracle import decoder, geometry, sampler
    lat = geometry.Lattice(L)
    syn, _, _ = sampler.sample(lat, p, SEED, np.arange(lo, lo + n), noise=noise)
    t0 = time.perf_counter()
    decoder.decode(L, syn, p, SWEEPS, SEED, chains_per_class=CHAINS, n_temps=K, burn=BURN,
                   syndrome_ids=np.arange(lo, lo + n), noise=noise,
                   scan=decoder.SCAN_RANDOM if random_scan else decoder.SCAN_COLOUR,
                   init_mode=decoder.INIT_MWPM if init == "mwpm" else decoder.INIT_MATCHING)
    return time.perf_counter() - t0


# the space-time workload's constants, shared by the bench and its oracle baseline
ST_L, ST_T, ST_P, ST_PM, ST_CHAINS, ST_SWEEPS = 7, 7, 0.02, 0.02, 4, 784


def _st_shard(job):
    """One worker: history id `hid` at sweeps // frac of the budget on the
    oracle; returns the seconds it took."""
    hid, frac = job
    here = os.path.dirname(os.path.abspath(__file__))
    if here not in sys.path:
        sys.path.insert(0, here)
    from oracle import geometry, spacetime as stm
    obs, _, _, _ = stm.sample(geometry.Lattice(ST_L), ST_P, ST_PM, ST_T, SEED, np.array([hid]))
    t0 = time.perf_counter()
    stm.decode(ST_L, obs, ST_P, ST_PM, ST_SWEEPS // frac, SEED, chains_per_class=ST_CHAINS,
               syndrome_ids=np.array([hid]))
    return time.perf_counter() - t0


def cpu_baseline_spacetime(workers):
    """The space-time oracle on one history per worker process at a quarter of
    the sweeps (its cost is linear in sweeps), scaled to the full budget."""
    frac = 4
    t0 = time.perf_counter()
    if workers == 1:
        _st_shard((0, frac))
    else:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            pool.map(_st_shard, [(w, frac) for w in range(workers)])
    dt = time.perf_counter() - t0
    return {"value": workers / (dt * frac), "unit": "histories/s", "cores": workers,
            "kind": "oracle", "host": host_core_note(workers),
            "sample": f"{workers} histories of the same workload at {ST_SWEEPS // frac} of its "
                      f"{ST_SWEEPS} sweeps, NumPy oracle in {workers} processes of one history "
                      f"each, {dt:.1f} s wall, time x{frac}"}

CPU_CORE_CAP = 16


def _affinity():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def host_cores():
    """Worker processes of the oracle baseline: the cores this process may run
    on, at most CPU_CORE_CAP (one GPU's share of a multi-GPU host)."""
    return max(1, min(CPU_CORE_CAP, _affinity()))


def host_core_note(workers):
    """What the host offered and what the baseline used."""
    return {"host_cpus": os.cpu_count(), "host_affinity": _affinity(), "cap": CPU_CORE_CAP,
            "cores_used": workers,
            "note": f"one forked process per core, capped at {CPU_CORE_CAP} cores (one GPU's "
                    "share of the host)"}


def cpu_baseline(n_sample, ns, noise=0, p=P, random_scan=False, workers=1, init="greedy"):
    """The oracle, as written, on a bounded sample of the same workload: one
    process per core, each decoding its own shard of n_sample syndromes.
    Worker processes are forked, so this runs before the GPU is touched."""
    jobs = [(w * n_sample, n_sample, noise, p, random_scan, init) for w in range(workers)]
    t0 = time.perf_counter()
    if workers == 1:
        _oracle_shard(jobs[0])
    else:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            pool.map(_oracle_shard, jobs)
    dt = time.perf_counter() - t0
    total = n_sample * workers
    model = "bit/phase flips q" if noise else "p"
    scan = ", random scan" if random_scan else ""
    return {"value": total / dt, "unit": "syndromes/s", "cores": workers, "kind": "oracle",
            "host": host_core_note(workers),
            "sample": f"{total} syndromes of the same workload (L=13, {model}={p}, 4x4 "
                      f"chains, 169 sweeps{scan}, {'exact enhanced-matching' if init == 'mwpm' else 'greedy matching'} "
                      f"starts), NumPy oracle in {workers} processes of "
                      f"{n_sample} syndromes each, {dt:.1f} s wall",
            "stabilizer_updates_per_s": total * 4 * CHAINS * K * (BURN + SWEEPS) * ns / dt}


if __name__ == "__main__":
    main()
