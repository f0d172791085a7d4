"""Benchmark of the FlashVAN hot path on one MI355X.

Workload: 3D Edwards-Anderson L = 10 (N = 1000 spins, periodic, Gaussian
bonds), transformer d_model = 128, 8 layers, 8 heads, batch 16384, beta = 1,
mask (window, prefix) derived from the lattice.  One step = one training step
of the method: KV-cached sampling of the batch, energies, F_q statistics,
REINFORCE weights, the hand-written backward and the Adam update.  Inputs
(couplings, parameters) are resident in HBM before timing starts.

Prints ONE JSON line.  value = spin samples per second through the full
training step in the headline precision (BF16_SPLIT: BF16 MFMA on split
operands with an FP16 K/V cache); FP32 is timed beside it.  After the timed
steps, 16 samples of the last timed step are re-scored by the FP64 oracle
(energy and teacher-forced ln q at the parameters they were drawn with); the
line carries the resulting |dF_q/N|, and value is null if it exceeds 1e-4.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Bytes moved per decode launch at this workload (FETCH_SIZE + WRITE_SIZE from two
# rocprofv3 --pmc runs, each scaled by the same counter's reading for a 1 GiB copy);
# the record with the commands is profiles/decode_ea3d_L10_hbm_counters.md.
# Set to None whenever decode_kernel changes until the counters are taken again.
DECODE_TRAFFIC_BYTES = 12385239098720
# learning rate: the paper's eta = 1e-3 reached by a linear warm-up over 300 steps
# (Methods, model configurations and training settings); the timed steps sit at
# the start of the warm-up
ETA, WARMUP_STEPS = 1e-3, 300


def warmup_lr(step):
    return ETA * min(1.0, step / WARMUP_STEPS)


def kv_bytes_per_sample(N, L, D, W, P, kv_elem):
    """Algorithmic K/V traffic of one sample's decode: every visible key and value
    read once per step and layer, plus the new key and value written."""
    R = min(W + 1, N - P)
    reads = 0
    for t in range(N):
        nvis = t + 1 if t < P else P + min(t - P + 1, R)
        reads += nvis
    return (reads * 2 * D + N * 2 * D) * kv_elem * L + N   # + spins


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# The paper's patched 3D EA L=10 model (SI, 3D EA settings): 2x2x2 patches, so
# 125 positions over a vocabulary of 256; d_token 32 + d_pos 96 = d_model 128,
# 2 heads, 2 layers, batch 2048; 0.179 s per training step on one H100.
PATCHED_3D = dict(L=10, D=3, d_model=128, d_token=32, n_heads=2, n_layers=2, batch=2048, paper_step_s=0.179)


def patched(args):
    """Training step of the paper's patched 3D EA L=10 model (sample tokens ->
    spins -> energies -> F_q -> REINFORCE weights -> token backward -> Muon), in
    split and FP32 mode, beside the paper's step time for the same workload."""
    import numpy as np
    import torch

    import paper_2606_22984_amd as fv
    from workloads import ModelConfig, ea_instance, init_params, workload
    from workloads.instances import patch_edges

    pc = PATCHED_3D
    wl = workload("ea3d_L10")
    inst = ea_instance(pc["L"], pc["D"], wl.instance_seed, wl.bonds)
    T, pi, pj = patch_edges(pc["L"], pc["D"])
    W, P = fv.derive_mask(T, pi, pj)
    cfg = ModelConfig(T, pc["d_model"], pc["n_layers"], pc["n_heads"], d_token=pc["d_token"],
                      vocab=2 ** (2 ** pc["D"])).with_mask(W, P)
    theta = init_params(cfg, wl.param_seed, "default")
    coup = fv.couplings(inst)
    sites = torch.as_tensor(fv.patch_sites(pc["L"], pc["D"]), device="cuda")
    B, beta, seed = pc["batch"], 1.0, 12345
    stream = torch.cuda.current_stream()
    out = {}
    for name, prec in (("bf16split", fv.FVAN_BF16_SPLIT), ("fp32", fv.FVAN_FP32)):
        m = fv.Model(cfg, B, prec, theta)
        stats = torch.zeros(4, dtype=torch.float64, device="cuda")
        for k in range(1, args.warmup + 1):
            m.train_step_tokens(coup, sites, beta, B, seed, k, stats, lr=warmup_lr(k), adam_lr=warmup_lr(k))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.warmup + 1, args.warmup + args.steps + 1):
            m.train_step_tokens(coup, sites, beta, B, seed, k, stats, lr=warmup_lr(k), adam_lr=warmup_lr(k))
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / args.steps
        # sampling alone, timed on the stream it runs on
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tok = torch.empty(B, T, dtype=torch.uint8, device="cuda")
        lq = torch.empty(B, dtype=torch.float32, device="cuda")
        m.sample_tokens(B, seed, 1, tok, lq)
        a.record(stream)
        m.sample_tokens(B, seed, 2, tok, lq)
        b.record(stream)
        torch.cuda.synchronize()
        st = stats.cpu().numpy()
        m.status()
        m.close()
        out[name] = {"ms_per_step": round(ms, 3), "samples_per_s": round(B / (ms * 1e-3), 1),
                     "sample_ms": round(a.elapsed_time(b), 3), "F_per_site": float(st[0])}
        progress(f"patched 3D step, {name}: {ms:.2f} ms per step")
    s = out["bf16split"]
    return {"metric": "training-step time, patched 3D EA L=10 (the paper's model and batch)",
            "value": s["ms_per_step"], "unit": "ms", "higher_is_better": False, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "dtype": "bf16-split-mfma+fp16-kv",
            "data": "synthetic: seeded Gaussian 3D EA instance and seeded random-init parameters",
            "config": {"workload": f"3D EA L={pc['L']} PBC, Gaussian J, 2x2x2 patches: {T} positions, vocabulary "
                                   f"{cfg.vocab}, d_model={cfg.d_model} (d_token {cfg.d_token}), "
                                   f"{cfg.n_layers} layers, {cfg.n_heads} heads, batch {B}, mask W={W} P={P}, "
                                   "REINFORCE + Muon"},
            "paper_step_ms": 1e3 * pc["paper_step_s"],
            "paper_hardware": "one NVIDIA H100 80GB, PyTorch 2.8 + FlashAttention-2, FP16 attention",
            "speedup_vs_paper": round(1e3 * pc["paper_step_s"] / s["ms_per_step"], 2),
            "precisions": out}


def single_workload(name, steps, warmup, optimizer="muon"):
    """Another single-model workload at its own sizes: the full training step
    (split and FP32) and sampling alone, with the decode's HBM roofline
    fraction (the K/V bytes it must read, per launch duration)."""
    import numpy as np
    import torch

    import paper_2606_22984_amd as fv
    from workloads import ea_instance, init_params, sk_instance, workload

    wl = workload(name)
    if wl.kind == "sk":
        inst = sk_instance(wl.size, wl.instance_seed)
        cfg = wl.model.full_causal()
    else:
        inst = ea_instance(wl.size, wl.dim, wl.instance_seed, wl.bonds)
        W, P = fv.derive_mask(inst.n, inst.edges_i, inst.edges_j)
        cfg = wl.model.with_mask(W, P)
    theta = init_params(cfg, wl.param_seed, "default")
    coup = fv.couplings(inst)
    B, beta, seed = wl.batch, float(wl.betas[0]), 777
    stream = torch.cuda.current_stream()
    out = {}
    for pname, prec in (("bf16split", fv.FVAN_BF16_SPLIT), ("fp32", fv.FVAN_FP32)):
        m = fv.Model(cfg, B, prec, theta)
        stats = torch.zeros(4, dtype=torch.float64, device="cuda")

        def step(k):
            if optimizer == "muon":
                m.train_step_muon(coup, beta, B, seed, k, stats, lr=warmup_lr(k), adam_lr=warmup_lr(k))
            else:
                m.train_step(coup, beta, B, seed, k, lr=warmup_lr(k), stats=stats)

        for k in range(1, warmup + 1):
            step(k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(warmup + 1, warmup + steps + 1):
            step(k)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        spins = torch.empty(B, cfg.n_spins, dtype=torch.int8, device="cuda")
        lq = torch.empty(B, dtype=torch.float32, device="cuda")
        m.sample(B, seed, 1, spins, lq)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for k in range(steps):
            m.sample(B, seed, 2 + k, spins, lq)
        b.record(stream)
        torch.cuda.synchronize()
        dec = a.elapsed_time(b) / steps
        m.status()
        m.close()
        kv = kv_bytes_per_sample(cfg.n_spins, cfg.n_layers, cfg.d_model, cfg.window, cfg.prefix,
                                 4 if prec == fv.FVAN_FP32 else 2) * B
        out[pname] = {"train_step_ms": round(ms, 3), "train_samples_per_s": round(B / (ms * 1e-3), 1),
                      "decode_ms": round(dec, 3), "sample_only_samples_per_s": round(B / (dec * 1e-3), 1),
                      "decode_hbm_frac": round(kv / (dec * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "F_per_site": float(stats[0].item())}
        progress(f"{name} {pname}: {ms:.1f} ms per step, decode {dec:.2f} ms")
    sp, fp = out["bf16split"], out["fp32"]
    return {"workload": f"{name}: N={cfg.n_spins}, d_model={cfg.d_model}, {cfg.n_layers} layers, {cfg.n_heads} heads, "
                        f"batch {B}, mask W={cfg.window} P={cfg.prefix}",
            "precisions": out,
            "speedup_vs_fp32": {"train_step": round(fp["train_step_ms"] / sp["train_step_ms"], 3),
                                "sampling": round(fp["decode_ms"] / sp["decode_ms"], 3)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--compare-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (2D EA L=16, SK N=512, the batched launch, the patched 3D step) "
                         "that the default line carries as extra keys")
    ap.add_argument("--optimizer", choices=("muon", "adam"), default="muon",
                    help="parameter update of the training step (muon: the paper's default)")
    ap.add_argument("--batched", action="store_true",
                    help="measure the batched workload instead: 64 2D EA instances (L in 16/24/32, +/-J) x 8 "
                         "temperatures, 1024 samples each, sampled + energies + F_q in one graph replay")
    ap.add_argument("--distill", action="store_true",
                    help="measure the 3D EA training step with local Monte Carlo refinement and the "
                         "self-distillation loss instead (Eq. loss2; --lmc-sweeps sweeps, likelihood weight --w)")
    ap.add_argument("--overlap", action="store_true",
                    help="time the overlap histogram of the 3D EA batch (16384 sampled configurations of 1000 "
                         "spins, all pairs) instead")
    ap.add_argument("--patched", action="store_true",
                    help="time the training step of the paper's patched 3D EA L=10 model instead (2x2x2 patches: "
                         "125 positions, vocabulary 256, d_model 128, 2 heads, 2 layers, batch 2048)")
    ap.add_argument("--lmc-sweeps", type=int, default=10)
    ap.add_argument("--w", type=float, default=0.1)
    ap.add_argument("--profile-decode", action="store_true",
                    help="no benchmark: one 1 GiB device copy (counter scale) then one decode launch at the "
                         "benchmark shape, for hardware-counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the path shards by samples, "
              "see the design notes for the multi-GPU layout", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2606_22984_amd as fv
    from workloads import ea_instance, init_params, workload

    torch.cuda.set_device(0)
    if args.batched:
        print(json.dumps(batched(args)))
        return
    wl = workload("ea3d_L10")
    inst = ea_instance(wl.size, wl.dim, wl.instance_seed, wl.bonds)
    W, P = fv.derive_mask(inst.n, inst.edges_i, inst.edges_j)
    cfg = wl.model.with_mask(W, P)
    theta = init_params(cfg, wl.param_seed, "default")
    B, beta, seed = wl.batch, 1.0, 12345
    N, L, D = cfg.n_spins, cfg.n_layers, cfg.d_model
    coup = fv.couplings(inst)

    if args.profile_decode:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)                       # reads and writes exactly 1 GiB
        m = fv.Model(cfg, B, fv.FVAN_BF16_SPLIT, theta)
        m.sample(B, seed, 1)
        torch.cuda.synchronize()
        print(json.dumps({"profile_decode": "done", "copy_bytes": 1 << 30,
                          "decode_algorithmic_bytes": kv_bytes_per_sample(N, L, D, W, P, 2) * B}))
        return

    if args.overlap:
        m = fv.Model(cfg, B, fv.FVAN_BF16_SPLIT, theta)
        spins, _ = m.sample(B, seed, 1)
        counts = torch.empty(N + 1, dtype=torch.int64, device="cuda")
        fv.overlap_histogram(spins, counts)
        stream = torch.cuda.current_stream()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.steps):
            fv.overlap_histogram(spins, counts)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / args.steps
        ops = 2.0 * B * B * N          # the full S S^T product the blocks of the upper triangle cover
        c = counts.cpu().numpy()
        q = 2.0 * np.arange(N + 1) / N - 1.0
        print(json.dumps({"metric": "overlap histogram of one batch (all sample pairs)", "value": round(ms, 3),
                          "unit": "ms", "higher_is_better": False, "n_gpus": 1, "steps": args.steps,
                          "config": {"workload": "3D EA L=10 model samples, batch 16384, N=1000"},
                          "pairs": int(c.sum()), "achieved_TOPS_int8": round(ops / 2 / (ms * 1e-3) / 1e12, 2),
                          "peak_TOPS_int8": 5000.0, "mean_abs_q": float((c * np.abs(q)).sum() / c.sum())}))
        return
    if args.distill:
        print(json.dumps(distill(args, cfg, theta, inst, coup, B, beta, seed, N)))
        return
    if args.patched:
        print(json.dumps(patched(args)))
        return

    def run(prec, steps, warmup):
        m = fv.Model(cfg, B, prec, theta)
        stream = torch.cuda.current_stream()
        spins = torch.empty(B, N, dtype=torch.int8, device="cuda")
        lq = torch.empty(B, dtype=torch.float32, device="cuda")
        E = coup.empty_energy(B)
        stats = torch.zeros(4, dtype=torch.float64, device="cuda")
        w = torch.empty(B, dtype=torch.float32, device="cuda")
        theta_snap = torch.empty_like(m.params)
        ev, ev_opt = [], []
        last = warmup + steps

        def step(k, timed):
            if k == last:
                theta_snap.copy_(m.params)       # the parameters the checked samples are drawn with
            if timed:
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                oa, ob = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
            m.sample(B, seed, k, spins, lq)
            if timed:
                b.record(stream)
                ev.append((a, b))
            fv.energy(coup, spins, E)
            fv.free_energy(E, lq, beta, N, stats[:2])
            fv.reinforce_weights(E, lq, beta, w)
            m.log_prob_backward(spins, w)
            if timed:
                oa.record(stream)
            if args.optimizer == "muon":
                m.muon_step(k, lr=warmup_lr(k), adam_lr=warmup_lr(k))
            else:
                m.adam_step(k, lr=warmup_lr(k))
            if timed:
                ob.record(stream)
                ev_opt.append((oa, ob))

        for k in range(1, warmup + 1):
            step(k, False)
        torch.cuda.synchronize()
        progress(f"precision {fv.PRECISION_NAMES[prec]}: warm-up done")
        t0 = time.perf_counter()
        for k in range(warmup + 1, warmup + steps + 1):
            step(k, True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        dec = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        st = stats.cpu().numpy()
        opt_ms = float(np.mean([a.elapsed_time(b) for a, b in ev_opt]))
        res = dict(ms_per_step=1e3 * wall / steps, samples_per_s=B * steps / wall, decode_ms=dec, optimizer_ms=opt_ms,
                   sample_only_samples_per_s=B / (dec * 1e-3), F_per_site=float(st[0]),
                   var_f=float(st[1]))
        progress(f"precision {fv.PRECISION_NAMES[prec]}: re-scoring {CHECK_SAMPLES} samples with the FP64 oracle")
        res["oracle_check"] = oracle_check(cfg, theta_snap.cpu().numpy(), inst, beta, spins, lq, E)
        m.close()
        del m
        torch.cuda.empty_cache()
        progress(f"precision {fv.PRECISION_NAMES[prec]}: {res['ms_per_step']:.1f} ms/step, decode {dec:.1f} ms")
        return res

    SPLIT, FP32 = fv.FVAN_BF16_SPLIT, fv.FVAN_FP32
    head = run(SPLIT, args.steps, args.warmup)
    others = {}
    if not args.no_compare:
        others["fp32"] = run(FP32, args.compare_steps, 1)
    kv_elem = 2
    bytes_launch = kv_bytes_per_sample(N, L, D, W, P, kv_elem) * B
    achieved = bytes_launch / (head["decode_ms"] * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": DECODE_TRAFFIC_BYTES,
            "kernel": "decode_kernel<128,2,16,false,32>", "algorithmic_bytes_per_launch": bytes_launch}

    extra = None
    if not args.no_extra:
        extra = {}
        for name in ("ea2d_L16", "sk512"):
            extra[name] = single_workload(name, 3, 1, args.optimizer)
        progress("batched workload")
        bargs = argparse.Namespace(steps=2)
        extra["ea2d_batched"] = batched(bargs)
        progress("patched 3D step")
        pargs = argparse.Namespace(steps=5, warmup=2)
        extra["ea3d_L10_patched"] = patched(pargs)

    cpu = None
    if not args.no_cpu_baseline:
        progress("timing the FP64 oracle on the host")
        cpu = cpu_baseline(cfg, theta, inst, beta, args.optimizer)

    ok = head["oracle_check"]["dF_per_site"] <= DF_TOL
    out = {
        "metric": "spin samples/sec + train-step ms, BF16 vs FP32, 1 GPU, at |dF/N|<=1e-4",
        "value": round(head["samples_per_s"], 2) if ok else None,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-split-mfma+fp16-kv",
        "data": "synthetic: seeded Gaussian 3D EA instance and seeded random-init parameters",
        "config": {"workload": "3D EA L=10 PBC (N=1000), Gaussian J, beta=1, d_model=128, 8 layers, 8 heads, "
                               "batch 16384, mask W=%d P=%d" % (W, P),
                   "global_batch": B, "seq_len": N, "parallelism": "none (1 GPU)"},
        "dF_per_site": head["oracle_check"]["dF_per_site"],
        "sample_only_samples_per_s": round(head["sample_only_samples_per_s"], 1),
        "decode_ms": round(head["decode_ms"], 2),
        "optimizer": args.optimizer,
        "optimizer_ms": round(head["optimizer_ms"], 3),
        "precisions": {"bf16split": _round(head), **{k: _round(v) for k, v in others.items()}},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if extra is not None:
        out["other_workloads"] = extra
    if "fp32" in others:
        out["speedup_vs_fp32"] = {
            "train_step": round(head["samples_per_s"] / others["fp32"]["samples_per_s"], 3),
            "sampling": round(head["sample_only_samples_per_s"] / others["fp32"]["sample_only_samples_per_s"], 3)}
    print(json.dumps(out))


def batched(args):
    """The batched workload: every (instance, beta) unit has its own model (random
    init), all units are sampled in one persistent launch, then energies and F_q
    statistics, all captured in one HIP graph."""
    import numpy as np
    import torch

    import paper_2606_22984_amd as fv
    from workloads import ea_instance, init_params, workload
    wl = workload("ea2d_batched")
    prec = fv.FVAN_BF16_SPLIT
    units = []
    for k in range(wl.n_instances):
        L = wl.sizes[k % len(wl.sizes)]
        inst = ea_instance(L, 2, wl.instance_seed + k, wl.bonds)
        W, P = fv.derive_mask(inst.n, inst.edges_i, inst.edges_j)
        cfg = wl.model.__class__(L * L, wl.model.d_model, wl.model.n_layers, wl.model.n_heads).with_mask(W, P)
        coup = fv.couplings(inst)
        for j, beta in enumerate(wl.betas):
            m = fv.Model(cfg, wl.batch, prec, init_params(cfg, wl.param_seed + 100 * k + j),
                         workspaces=fv.WS_SAMPLER)
            units.append(dict(model=m, couplings=coup, beta=beta, batch=wl.batch, seed=7, stream_id=k * 16 + j))
    progress(f"batched: {len(units)} units built")
    t0 = time.perf_counter()
    g = fv.Group(units)
    torch.cuda.synchronize()
    shape = g.launch_shape()
    progress(f"batched: group created in {time.perf_counter() - t0:.1f} s, launch shape {shape}")
    g.run_graph()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(1, args.steps)
    a.record(stream)
    for _ in range(reps):
        g.run_graph()
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    total = sum(u["batch"] for u in units)
    kv = sum(kv_bytes_per_sample(u["model"].cfg.n_spins, u["model"].cfg.n_layers, u["model"].cfg.d_model,
                                 u["model"].cfg.window, u["model"].cfg.prefix, 2) * u["batch"] for u in units)
    achieved = kv / (ms * 1e-3) / 1e9
    return {"metric": "batched sampling + energy + F_q (spin samples/s)", "value": round(total / (ms * 1e-3), 1),
            "unit": "samples/s", "ms_per_launch": round(ms, 2), "units": len(units), "samples_per_launch": total,
            "launch_shape": shape,
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_launch": kv},
            "dtype": "bf16-split-mfma+fp16-kv",
            "config": {"workload": "64 2D EA instances (L=16/24/32 round-robin, +/-J) x 8 betas in [0.2, 3.0], "
                                   "d_model=64, 4 layers, 4 heads, 1024 samples per unit, one graph replay"}}


def distill(args, cfg, theta, inst, coup, B, beta, seed, N):
    """The 3D EA training step of the paper's low-temperature procedure: sample,
    refine by checkerboard Metropolis, teacher-forced log q of the refined
    samples, Eq. (loss2) weights, backward, Muon (BF16_SPLIT)."""
    import numpy as np
    import torch
    import paper_2606_22984_amd as fv
    g = fv.lmc_graph(inst, args.lmc_sweeps)
    m = fv.Model(cfg, B, fv.FVAN_BF16_SPLIT, theta)
    stream = torch.cuda.current_stream()
    stats = torch.zeros(4, dtype=torch.float64, device="cuda")
    for k in range(1, args.warmup + 1):
        m.train_step_distill(coup, g, beta, args.w, B, seed, k, stats, lr=warmup_lr(k), adam_lr=warmup_lr(k))
    torch.cuda.synchronize()
    progress("distillation step: warm-up done")
    t0 = time.perf_counter()
    for k in range(args.warmup + 1, args.warmup + args.steps + 1):
        m.train_step_distill(coup, g, beta, args.w, B, seed, k, stats, lr=warmup_lr(k), adam_lr=warmup_lr(k))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the refinement kernel alone, on the step's own samples, timed on its stream
    spins, _ = m.sample(B, seed, 1)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fv.lmc_refine(g, spins, beta, seed, 0x80000001)
    a.record(stream)
    fv.lmc_refine(g, spins, beta, seed, 0x80000002)
    b.record(stream)
    torch.cuda.synchronize()
    lmc_ms = a.elapsed_time(b)
    updates = B * N * args.lmc_sweeps
    st = stats.cpu().numpy()
    m.close()
    return {"metric": "spin samples/sec + train-step ms, 3D EA training step with local Monte Carlo refinement "
                      "and self-distillation (Eq. loss2)",
            "value": round(B * args.steps / wall, 2), "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(1e3 * wall / args.steps, 2), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "bf16-split-mfma+fp16-kv",
            "data": "synthetic: seeded Gaussian 3D EA instance and seeded random-init parameters",
            "config": {"workload": "3D EA L=10 PBC (N=1000), Gaussian J, beta=1, d_model=128, 8 layers, 8 heads, "
                                   "batch 16384, %d checkerboard Metropolis sweeps, w=%g" % (args.lmc_sweeps, args.w),
                       "global_batch": B, "seq_len": N, "parallelism": "none (1 GPU)"},
            "lmc_ms": round(lmc_ms, 3), "lmc_spin_updates_per_s": round(updates / (lmc_ms * 1e-3), 1),
            "F_per_site_raw": float(st[0])}


def _round(d):
    return {k: (round(v, 6) if isinstance(v, float) else v) for k, v in d.items()}


CHECK_SAMPLES, DF_TOL = 16, 1e-4


def oracle_check(cfg, theta, inst, beta, spins, lq, E):
    """|F_q/N (GPU) - F_q/N (FP64 oracle)| over CHECK_SAMPLES samples spread over the
    batch: the oracle re-evaluates the energy and the teacher-forced ln q of the
    GPU's own samples at the parameters they were drawn with."""
    import numpy as np
    from oracle import estimator, network as net, physics
    B = spins.shape[0]
    rows = np.linspace(0, B - 1, CHECK_SAMPLES).round().astype(np.int64)
    sp = spins.cpu().numpy()[rows]
    lq_gpu = lq.cpu().numpy()[rows].astype(np.float64)
    E_gpu = E.cpu().numpy()[rows].astype(np.float64)
    E_ref = physics.energy_edges(sp, inst.edges_i, inst.edges_j, inst.J.astype(np.float32).astype(np.float64))
    lq_ref = net.log_q(net.as_theta(theta), cfg, sp, chunk=4).numpy()
    f_gpu, _ = estimator.free_energy_stats(E_gpu, lq_gpu, beta, cfg.n_spins)
    f_ref, _ = estimator.free_energy_stats(E_ref, lq_ref, beta, cfg.n_spins)
    return {"samples": CHECK_SAMPLES, "dF_per_site": float(abs(f_gpu - f_ref)),
            "max_site_dlogq": float(np.max(np.abs(lq_gpu - lq_ref)) / cfg.n_spins),
            "max_dE_per_site": float(np.max(np.abs(E_gpu - E_ref)) / cfg.n_spins)}


def cpu_baseline(cfg, theta, inst, beta, optimizer, n_samples=8):
    """The FP64 oracle (as it stands) running the same training step on a bounded
    sample: KV-cached sampling of n_samples, energies, REINFORCE weights, the
    reverse-mode gradient and the parameter update.  Throughput in samples/s of
    that step."""
    import numpy as np
    import torch
    from oracle import estimator, muon, physics, sampler
    t0 = time.perf_counter()
    spins, lq, _ = sampler.kv_sample(theta, cfg, n_samples, 12345, 1)
    E = physics.energy_edges(spins, inst.edges_i, inst.edges_j, inst.J)
    estimator.free_energy_stats(E, lq, beta, cfg.n_spins)
    g = estimator.reinforce_gradient(theta, cfg, spins, E, lq, beta)
    z = np.zeros_like(g)
    if optimizer == "muon":
        muon.muon_update(theta, g, z, z, 1, cfg, warmup_lr(1), adam_lr=warmup_lr(1))
    else:
        estimator.adam_update(theta, g, z, z, 1, warmup_lr(1))
    dt = time.perf_counter() - t0
    return {"value": round(n_samples / dt, 5), "unit": "samples/s", "cores": torch.get_num_threads(),
            "kind": "oracle", "sample": f"{n_samples} samples of the same workload through one FP64 training step "
                                        f"(sampling, energy, estimator, gradient, {optimizer} update): {dt:.1f} s"}


if __name__ == "__main__":
    main()
