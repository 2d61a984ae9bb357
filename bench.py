"""Benchmark of the culled N-D Gaussian mixture fwd+bwd step on one MI355X.

    python bench.py [--gpus 1] [--steps 10] [--warmup 3] [--workload 10d-fwdbwd]

One step is the whole hot path on one batch, every stage a libngd call:
  update (float64 inversion of every factor) -> cull build (projections,
  sort, tiles, interval test, candidate lists) -> forward -> L2 loss and its
  gradient -> backward (gradients of mean, factor, weight, colour).
Inputs are resident in HBM before timing starts.  `value` is dense-equivalent
Gaussian-query evaluations per second of the step: Q*K / (time per step).

Prints one JSON line (rank 0).  Also times the plain float32 dense direct-sum
kernel (forward and backward, no culling) once for the speedup, and the
float64 CPU oracle on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Published dense FP32 vector peak without packed-FP32 instructions: the
# library is built with those disabled, so 157.3 (packed) is out of reach.
FP32_VALU_PEAK_TFLOPS = 78.6
BF16_MFMA_PEAK_TFLOPS = 2500.0  # published dense BF16 matrix peak
TRAFFIC_FILES = dict(fp32=os.path.join(ROOT, "profiles", "forward_10d_traffic.json"),
                     bf16_mfma=os.path.join(ROOT, "profiles", "forward_mfma_10d_traffic.json"))
KERNEL_SRC = os.path.join(ROOT, "paper_2405_20067_amd", "csrc", "eval.hip")
MFMA_SRC = os.path.join(ROOT, "paper_2405_20067_amd", "csrc", "eval_mfma.hip")


def stage_flops(n: int):
    """float32 flops one lane spends on each stage of a (query, Gaussian) pair
    in the forward kernel: rows [a, b) of y = S'(x - m) cost, per row r,
    1 subtraction, 1 multiply + r fmas, and 1 fma into the squared norm;
    the kept pair adds exp2 and 3 fmas.  Stage boundaries 3 and 6."""
    k1, k2 = min(3, n), min(6, n)
    rows = lambda a, b: sum(1 + 1 + 2 * r + 2 for r in range(a, b))
    return rows(0, k1), rows(k1, k2), rows(k2, n), 1 + 6


def fp32_pair_flops(n: int) -> int:
    """Algorithmic float32 flops of one (query, Gaussian) pair of the direct
    sum: n subtractions, the triangular product y = S'(x - m) (n(n+1)/2
    fmas), the squared norm (n fmas), exp2 and the 3 colour fmas -- 38, 66
    and 146 at n = 4, 6, 10."""
    return 3 * n + n * (n + 1) + 6


def mfma_pair_flops(n: int) -> int:
    """Algorithmic matrix-core flops of one (query, candidate) pair: one
    multiply-add per quadratic feature (1 + n + n(n+1)/2; 132 flops at
    n = 10)."""
    return 2 * (1 + n + n * (n + 1) // 2)


def source_hash(*paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def setup(workload: str):
    import torch
    from paper_2405_20067_amd import inputs
    w = inputs.WORKLOADS[workload]
    t0 = time.time()
    mix = inputs.workload_mixture(w)
    tgt = inputs.workload_mixture(w, k=w.k_target, seed=inputs.SEED_TARGET) if w.k_target else None
    x = inputs.gen_workload_queries(w, mixtures=[m for m in (mix, tgt) if m is not None])
    proj = inputs.gen_projections(w.n, 16, inputs.SEED_PROJ)
    log(f"generated {workload}: n={w.n} k={w.k} q={w.q} in {time.time() - t0:.1f}s")
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    dev = dict(mean=d(mix["mean"]), factor=d(mix["factor"]), weight=d(mix["weight"]),
               colour=d(mix["colour"]), x=d(x))
    return w, mix, tgt, x, proj, dev


def targets(w, tgt, dev, proj):
    """Values of the hidden target mixture at the queries (workload input,
    computed once before timing with the library's culled forward)."""
    import torch
    from paper_2405_20067_amd import ngd
    if tgt is None:
        return torch.zeros((w.q, 3), dtype=torch.float32, device="cuda")
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    mt = ngd.Mixture(w.n, tgt["mean"].shape[0])
    mt.update(d(tgt["mean"]), d(tgt["factor"]), d(tgt["weight"]), d(tgt["colour"]))
    ct = ngd.Cull().build(mt, dev["x"], proj)
    t = ngd.eval_mixture(mt, ct, dev["x"])
    torch.cuda.synchronize()
    return t


def cpu_baseline(w, mix, x, budget_s: float, threads: int = 0):
    """The float64 oracle, fwd (direct sum over all K) + bwd (gradient of all
    K Gaussians) on a sample of queries, timed on this host with `threads`
    OpenMP threads (0: all the library starts with)."""
    import oracle
    from paper_2405_20067_amd import inputs
    full = oracle.threads() if not hasattr(cpu_baseline, "full") else cpu_baseline.full
    cpu_baseline.full = full
    oracle.set_threads(threads if threads > 0 else full)
    rng = np.random.default_rng(12345)
    g_all = inputs.gen_grad_out(w.q, seed=77)
    def run(nq):
        idx = rng.choice(w.q, nq, replace=False)
        xs, gs = x[idx], g_all[idx]
        t0 = time.perf_counter()
        oracle.eval_mixture(mix["mean"], mix["factor"], mix["weight"], mix["colour"], xs)
        t1 = time.perf_counter()
        oracle.grad(mix["mean"], mix["factor"], mix["weight"], mix["colour"], xs, gs)
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1
    # probe with enough queries to keep every core busy, then scale the
    # sample to the time budget
    used = int(oracle.threads())
    probe = max(4, min(256, 16 * used))
    a, b = run(probe)
    nq = int(max(probe, min(w.q, probe * budget_s / max(a + b, 1e-6))))
    tf, tb = run(nq)
    oracle.set_threads(full)
    pairs = nq * w.k
    return dict(value=pairs / (tf + tb), unit="Gaussian-query evals/s",
                cores=used, kind="oracle",
                sample=f"{nq} of the {w.q} queries (seeded), every one of the {w.k} "
                       f"Gaussians: float64 forward sum ({tf:.1f}s) + gradient of all "
                       f"Gaussians over those queries ({tb:.1f}s), {used} thread(s)",
                fwd_s=tf, bwd_s=tb, pairs=pairs)


def fit_bench(steps: int, precision_name: str, phase: int = 300, lr: float = 1e-3,
              lr_alpha: float = 3e-2, lr_child: float | None = None, init_scale: float = 0.7,
              per_component: float = 8, child_alpha: float = 1e-4, child_jitter: float = 1e-2,
              checkpoint: str | None = None, target_kind: str = "coarse",
              detail_sub: int = 16, detail_narrow: float = 0.35, adam_eps: float = 1e-15):
    """The 10-D fitting loop (Adam, children from the second phase,
    materialised above t = 0.01): K starts at 32,768 Gaussians and may grow
    to 524,288; 2^21 queries near the hidden K=4,096 target mixture and
    uniform, their target values computed once.  The start stands in for an
    initialisation from the data: `per_component` Gaussians per target
    component (below 1: one Gaussian on each of that fraction of the
    components, a seeded subset), means drawn from that component (with
    one per component: its mean), factors scaled by
    `init_scale` (below 1: narrower than the target, so the start
    under-covers it and children have room to grow), brightness
    1/per_component, colours random.  Every step is timed; set-up (query
    pool, targets, handles) is not.  `checkpoint`: the fit's state is saved
    there at the end.  target_kind "detail": the hidden target is the
    K=4,096 mixture with each component replaced by 16 narrower ones
    (`detail_sub` components of factors `detail_narrow` times the coarse
    one's: K_t = 65,536 by default, inputs.gen_detailed_mixture) while the
    start stays on the coarse components, so that the fit has to add
    Gaussians to reach it."""
    import torch
    from paper_2405_20067_amd import inputs, ngd
    from paper_2405_20067_amd.fit import Fit
    w = inputs.WORKLOADS["10d-fwdbwd"]
    k0, q, max_k = 32768, 1 << 21, 524288
    tgt = inputs.workload_mixture(w, k=w.k_target, seed=inputs.SEED_TARGET)
    rng = np.random.default_rng(inputs.SEED_MIXTURE)
    if per_component >= 1:
        rep = int(per_component)
        src = np.repeat(np.arange(w.k_target), rep)
    else:
        rep = 1
        src = np.sort(rng.choice(w.k_target, max(1, round(per_component * w.k_target)),
                                 replace=False))
    k0 = src.size
    lfull = np.zeros((k0, w.n, w.n))
    r, c = np.tril_indices(w.n)
    lfull[:, r, c] = tgt["factor"][src]
    z = rng.standard_normal((k0, w.n)) if rep > 1 else np.zeros((k0, w.n))
    mix = dict(mean=tgt["mean"][src] + np.einsum("kij,kj->ki", lfull, z),
               factor=init_scale * tgt["factor"][src], weight=tgt["weight"][src] / rep,
               colour=rng.uniform(0.05, 0.95, (k0, 3)))
    mix = {a: np.ascontiguousarray(v, np.float32) for a, v in mix.items()}
    hidden = inputs.gen_detailed_mixture(tgt, sub=detail_sub, narrow=detail_narrow) \
        if target_kind == "detail" else tgt
    x = inputs.gen_workload_queries(w, q=q, mixtures=[hidden])
    proj = inputs.gen_projections(w.n, 16, inputs.SEED_PROJ)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    dev = dict(x=d(x))
    target = targets(w, hidden, dev, proj)
    prec = ngd.BF16_MFMA if precision_name == "bf16_mfma" else ngd.FP32
    fit = Fit(d(mix["mean"]), d(mix["factor"]), d(mix["weight"]), d(mix["colour"]), lr=lr,
              lr_alpha=lr_alpha, lr_child=lr_child, phase=phase, max_k=max_k, precision=prec,
              child_alpha=child_alpha, child_jitter=child_jitter, adam_eps=adam_eps)
    log(f"fit: n={w.n} k0={k0} q={q} steps={steps} phase={phase} lr={lr}/{lr_alpha} "
        f"{precision_name}")
    ks, losses = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        loss = fit.step(dev["x"], target, proj)
        if i == 0 or (i + 1) % phase == 0 or i + 1 == steps:
            losses.append((i + 1, float(loss[0])))   # synchronises: a few times per run
            ks.append((i + 1, fit.k))
            rl = fit.refine_log[-1] if fit.refine_log and fit.refine_log[-1][0] == i + 1 \
                else None
            log(f"fit step {i + 1}: loss {losses[-1][1]:.5g}, K {fit.k}" +
                (f"; refinement: {rl[1]} materialised, brightest child {rl[2]:.3g}, "
                 f"{rl[3]} above t/10" if rl else ""))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / max(steps, 1)
    if checkpoint:
        fit.save(checkpoint)
    print(json.dumps(dict(
        metric="10-D fitting loop time per step (update, cull, fwd, loss, bwd, Adam, refinement)",
        value=ms, unit="ms/step", n_gpus=1, steps=steps, warmup=0, ms_per_step=ms,
        higher_is_better=False, scaling="weak", vs_baseline=None,
        dtype="bf16+f32" if prec == ngd.BF16_MFMA else "f32", data="synthetic",
        config=dict(workload="10d-fit", n=w.n, k_start=k0, k_max=max_k, q=q, phase=phase,
                    lr=lr, lr_alpha=lr_alpha, lr_child=fit.lr_child, threshold=fit.threshold,
                    loss="l2",
                    precision=precision_name,
                    init=(f"{rep} per target component" if per_component >= 1 else
                          f"one on {k0} of the {w.k_target} target components") +
                         f", factors x{init_scale}",
                    child_alpha=child_alpha, child_jitter=child_jitter, adam_eps=adam_eps,
                    target=target_kind, k_target=int(hidden["mean"].shape[0])),
        initial_loss=losses[0][1], final_loss=losses[-1][1], loss_trajectory=losses,
        k_trajectory=ks, refinements=[dict(step=a, materialised=b, brightest=round(m, 6),
                                           above_tenth=t) for a, b, m, t in fit.refine_log])),
        flush=True)


def sweep_bench(reps: int = 5, sample: int = 4096):
    """The cull's thresholds on the 10-D workload (Q = 2^20, K = 2^18): for
    each (tau, tile) the candidate fraction of the tile x Gaussian pairs,
    the cull build and both forwards' times (median of reps), and the
    normwise error of the culled FP32 forward against the float64 oracle's
    full sum on a seeded sample of queries.  tau = exp(-4.5) is the 3-sigma
    cut."""
    import torch
    from paper_2405_20067_amd import inputs, ngd
    w, mix, tgt, x, proj, dev = setup("10d-fwdbwd")
    m = ngd.Mixture(w.n, w.k)
    m.update(dev["mean"], dev["factor"], dev["weight"], dev["colour"])
    idx = torch.from_numpy(np.sort(np.random.default_rng(inputs.SEED_QUERIES).choice(
        w.q, sample, replace=False))).to("cuda")
    # the reference: the float64 oracle's full sum over all K at the sample
    import oracle
    t1 = time.perf_counter()
    dense = torch.from_numpy(oracle.eval_mixture(mix["mean"], mix["factor"], mix["weight"],
                                                 mix["colour"], x[idx.cpu().numpy()])).to("cuda")
    log(f"sweep: oracle on {sample} queries in {time.perf_counter() - t1:.1f}s")
    s3 = math.exp(-4.5)
    grid = [(t, 256) for t in (1e-2, s3, 1e-3, 1e-4, 1e-5, 1e-6)] + \
           [(1e-4, t) for t in (64, 128, 512, 1024)]

    def med(fn):
        out = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            out.append(a.elapsed_time(b))
        return float(np.median(out))

    rows = []
    for tau, tile in grid:
        p = ngd.default_params()
        p.tau, p.tile = tau, tile
        c = ngd.Cull().build(m, dev["x"], proj, p)
        f = ngd.eval_mixture(m, c, dev["x"])
        torch.cuda.synchronize()
        st = c.stats()
        err = float((f[idx].double() - dense).abs().max() / dense.abs().max())
        row = dict(tau=tau, tile=tile, candidates=st["total"],
                   fraction=st["total"] / max(st["ntiles"] * w.k, 1),
                   cull_ms=med(lambda: c.build(m, dev["x"], proj, p)),
                   fwd_fp32_ms=med(lambda: ngd.eval_mixture(m, c, dev["x"], out=f)),
                   fwd_bf16_ms=med(lambda: ngd.eval_mixture(m, c, dev["x"], out=f,
                                                            precision=ngd.BF16_MFMA)),
                   err_fp32=err)
        log(f"sweep tau={tau:.4g} tile={tile}: {row['fraction']:.4%} of pairs, cull "
            f"{row['cull_ms']:.3f} ms, fwd {row['fwd_fp32_ms']:.3f} / {row['fwd_bf16_ms']:.3f} "
            f"ms, err {err:.2e}")
        rows.append(row)
    print(json.dumps(dict(
        metric="cull thresholds on the 10-D workload: candidate fraction, cull and forward "
               "time, error against the float64 oracle",
        unit="ms", n_gpus=1, data="synthetic", dtype="f32 / bf16+f32",
        config=dict(workload="10d-fwdbwd", n=w.n, k=w.k, q=w.q, n_proj=16,
                    error_sample=sample, reps=reps),
        rows=rows)), flush=True)


def forward_roofline(w, m, cull, dev, prec, name, t, cand_pairs):
    """Roofline of one path's culled forward kernel.  `t` is its launch time
    (median over the timed steps, HIP events on the library's stream).

    FP32 (ALU bound): the float32 flops the kernel executes, counted by the
    same kernel in a counting mode on the same cull (its staged checks skip
    most of the candidate pairs' rows), against the non-packed FP32 peak.
    BF16-MFMA (matrix-core bound): the algorithmic contraction, one
    multiply-add per quadratic feature for every (query, candidate) pair the
    cull kept, against the dense BF16 peak; what the kernel executes (three
    split products, padded k-steps) is reported beside it."""
    from paper_2405_20067_amd import ngd
    cnt = ngd.eval_stats(m, cull, dev["x"], precision=prec)
    f1, f2, f3, f4 = stage_flops(w.n)
    valu = 64 * (f1 * cnt["filtered"] + f2 * cnt["pass1"] + f3 * cnt["pass2"]
                 + f4 * cnt["kept"])
    src = (KERNEL_SRC,) if name == "fp32" else (MFMA_SRC, KERNEL_SRC)
    traffic = None
    tf = TRAFFIC_FILES[name]
    if os.path.exists(tf):
        tr = json.load(open(tf))
        if tr.get("source_sha256_16") == source_hash(*src) and tr.get("workload") == w.name:
            traffic = tr.get("hbm_bytes_per_launch")
    if name == "fp32":
        a = valu / t / 1e12
        return dict(bound="alu", kernel="forward: k_eval_items + k_eval_reduce (ngd_eval)",
                    achieved=a, peak=FP32_VALU_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=a / FP32_VALU_PEAK_TFLOPS, traffic=traffic,
                    units=dict(group_candidate_pairs=cnt,
                               flops_per_lane_per_stage=[f1, f2, f3, f4],
                               lanes_per_pair=64, flops_per_launch=valu,
                               algorithmic_flops_per_pair=fp32_pair_flops(w.n),
                               candidate_pairs=cand_pairs,
                               launch_ms=t * 1e3))
    nf = 1 + w.n + w.n * (w.n + 1) // 2
    ks = 1 + (w.n * (w.n + 1) // 2 + 15) // 16
    alg = cand_pairs * mfma_pair_flops(w.n)
    a = alg / t / 1e12
    return dict(bound="mfma", kernel="forward: k_mfma_filter (ngd_eval, NGD_BF16_MFMA; "
                                     "its once-per-build records timed apart as "
                                     "eval_prepare)",
                achieved=a, peak=BF16_MFMA_PEAK_TFLOPS, unit="TFLOP/s",
                frac=a / BF16_MFMA_PEAK_TFLOPS, traffic=traffic,
                units=dict(candidate_pairs=cand_pairs, features=nf,
                           flops_per_pair=mfma_pair_flops(w.n),
                           flops_per_launch=alg, launch_ms=t * 1e3,
                           group_candidate_pairs=cnt,
                           executed_split_flops=cnt["examined"] * 64 * nf * 2 * 3,
                           executed_padded_flops=cnt["examined"] * 64 * ks * 16 * 2 * 3,
                           executed_split_tflops=cnt["examined"] * 64 * nf * 6 / t / 1e12,
                           fp32_survivor_flops=valu,
                           fp32_survivor_tflops=valu / t / 1e12))


def run_workload(name: str, args, precisions, with_dense: bool, steps: int, warmup: int,
                 profile_copy: bool = False):
    """Times `steps` steps of one workload (after `warmup` untimed ones) for
    each forward precision, and returns the workload's record: per path the
    step time, its stages, dense-equivalent evals/s and the forward's
    roofline; the cull's statistics; the dense float32 direct sum once."""
    import torch
    from paper_2405_20067_amd import ngd
    w, mix, tgt, x, proj, dev = setup(name)
    target = targets(w, tgt, dev, proj) if w.backward else None

    m = ngd.Mixture(w.n, w.k)
    cull = ngd.Cull()
    params = ngd.default_params()
    grads = (torch.empty((w.k, w.n), device="cuda"),
             torch.empty((w.k, w.n * (w.n + 1) // 2), device="cuda"),
             torch.empty((w.k,), device="cuda"), torch.empty((w.k, 3), device="cuda"))
    f = torch.empty((w.q, 3), device="cuda")
    loss = torch.empty((1,), device="cuda")
    gout = torch.empty((w.q, 3), device="cuda")
    # eval_prepare: what the forward derives once per cull build (the BF16
    # path's coefficient records; nothing for FP32), timed apart so that
    # `forward` is the forward kernel alone
    stages = ["update", "cull_build", "eval_prepare", "forward", "loss", "backward"]

    def step(prec, ev=None):
        def mark(i):
            if ev is not None:
                ev[i].record()
        mark(0)
        m.update(dev["mean"], dev["factor"], dev["weight"], dev["colour"])
        mark(1)
        if w.culled:
            cull.build(m, dev["x"], proj, params)
        mark(2)
        c = cull if w.culled else None
        if w.culled:
            ngd.eval_prepare(m, c, dev["x"], precision=prec)
        mark(3)
        ngd.eval_mixture(m, c, dev["x"], out=f, precision=prec)
        mark(4)
        if w.backward:
            ngd.l2_loss(f, target, loss=loss, grad=gout)
        mark(5)
        if w.backward:
            ngd.eval_backward(m, c, dev["x"], gout, grads=grads, precision=prec)
        mark(6)

    def timed(prec):
        for _ in range(warmup):
            step(prec)
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(stages) + 1)]
               for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step(prec, evs[i])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per_stage = {s: [] for s in stages}
        for e in evs:
            for j, s in enumerate(stages):
                per_stage[s].append(e[j].elapsed_time(e[j + 1]))
        return wall * 1e3 / steps, {s: float(np.median(v)) for s, v in per_stage.items()}

    precs = {"fp32": ngd.FP32, "bf16_mfma": ngd.BF16_MFMA}
    chosen = list(precisions) if w.culled else ["fp32"]
    paths = {}
    for pname in chosen:
        ms, sm = timed(precs[pname])
        paths[pname] = dict(ms_per_step=ms, value=w.q * w.k / (ms * 1e-3), stages_ms=sm)
        log(f"{name} {pname}: step {ms:.3f} ms; stages " +
            ", ".join(f"{s} {v:.3f}" for s, v in sm.items()))
    head = min(paths, key=lambda k: paths[k]["ms_per_step"])

    st = cull.stats() if w.culled else dict(total=w.k, ntiles=1, max_per_tile=w.k)
    tile = params.tile
    if w.culled:
        # every tile but the last holds `tile` queries; the workloads' query
        # counts are multiples of the tile, so candidates x tile is exact
        assert w.q % tile == 0
        cand_pairs = st["total"] * tile
    else:
        cand_pairs = w.q * w.k
    log(f"{name} headline {head}: step {paths[head]['ms_per_step']:.3f} ms"
        f"; candidates {st['total']} ({st['total'] / max(st['ntiles'] * w.k, 1):.4%} of "
        f"tile x Gaussian pairs), max/tile {st['max_per_tile']}")

    dense = None
    if with_dense:
        # the plain float32 direct-sum kernels, no culling, same inputs
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        ngd.eval_mixture(m, None, dev["x"], out=f)
        e[1].record()
        if w.backward:
            ngd.eval_backward(m, None, dev["x"], gout, grads=grads)
        e[2].record()
        torch.cuda.synchronize()
        dense = dict(forward_ms=e[0].elapsed_time(e[1]), backward_ms=e[1].elapsed_time(e[2]))
        if w.culled:
            # the culled side pays for its cull build and prepare every step
            for pname, pth in paths.items():
                sm = pth["stages_ms"]
                culled = (sm["cull_build"] + sm["eval_prepare"] + sm["forward"] +
                          sm["backward"])
                pth["speedup_vs_dense"] = (dense["forward_ms"] + dense["backward_ms"]) / culled
            dense["speedup_vs_dense"] = paths[head]["speedup_vs_dense"]
        log(f"{name} dense fp32 direct sum: fwd {dense['forward_ms']:.1f} ms, "
            f"bwd {dense['backward_ms']:.1f} ms")

    fl = fp32_pair_flops(w.n)
    for pname in paths:
        t = paths[pname]["stages_ms"]["forward"] * 1e-3
        if not w.culled:
            a = cand_pairs * fl / t / 1e12
            paths[pname]["roofline"] = dict(
                bound="alu", kernel="forward: k_eval_dense (ngd_eval, no cull)", achieved=a,
                peak=FP32_VALU_PEAK_TFLOPS, unit="TFLOP/s", frac=a / FP32_VALU_PEAK_TFLOPS,
                traffic=None,
                units=dict(pairs=cand_pairs, flops_per_pair=fl, launch_ms=t * 1e3))
        else:
            paths[pname]["roofline"] = forward_roofline(w, m, cull, dev, precs[pname], pname, t,
                                                        cand_pairs)
        r = paths[pname]["roofline"]
        log(f"{name} {pname} forward: {r['achieved']:.1f} {r['unit']} ({r['bound']}, "
            f"frac {r['frac']:.3f})")
    if profile_copy:
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 268435456 bytes read, 268435456 bytes written")
        del src, dst

    rec = dict(
        workload=w.name, description=w.description, n=w.n, k=w.k, q=w.q,
        k_target=w.k_target, near_frac=w.near_frac, n_proj=params.n_proj,
        tau=params.tau, tile=params.tile,
        tiling="k-d" if params.tiling == 0 else "morton",
        head=head, value=paths[head]["value"], ms_per_step=paths[head]["ms_per_step"],
        stages_ms=paths[head]["stages_ms"], paths=paths,
        cull=dict(candidates=st["total"], ntiles=st["ntiles"], max_per_tile=st["max_per_tile"],
                  candidate_pairs=cand_pairs,
                  survivor_fraction=st["total"] / max(st["ntiles"] * w.k, 1)),
        candidate_pairs_per_s_forward=cand_pairs / (
            (paths[head]["stages_ms"]["eval_prepare"] + paths[head]["stages_ms"]["forward"])
            * 1e-3),
        dense_fp32=dense)
    return rec, (w, mix, x)


# the workloads of the other configurations, timed after the headline one
# and reported beside it in the same line
OTHER_WORKLOADS = ("4d-dense", "6d-culled", "10d-uniform", "10d-4m")


def image_bench(reps: int = 5, sample: int = 2048, width: int = 800, k: int = 262144):
    """The cull on image-coherent queries (the paper's setting, Sec. 3.2): a
    synthetic 10-D G-buffer of width x width pixels laid out in 16 x 16 pixel
    tiles, a K-Gaussian mixture sitting on its features.  For each tiling
    (the image's own 16 x 16 tiles, the k-d order, the Morton order) and
    threshold (tau = 1e-4 and the paper's 3 sigma): the candidate fraction,
    the cull build and both forwards (median of reps), and the normwise error
    of the culled FP32 forward against the float64 oracle's full sum on a
    seeded sample of pixels; the dense FP32 forward for the speedup.  Then
    the global-conditioning case: with every input but the position constant
    over the image, the mixture conditioned on those values (a 3-D mixture,
    ngd_mixture_condition) against the 10-D path on the same pixels."""
    import torch
    import oracle
    from paper_2405_20067_amd import inputs, ngd
    n = 10
    t0 = time.time()
    x = inputs.gen_gbuffer(width, width)
    mix = inputs.gen_mixture_on(x, k, (10.0, 200.0), 5.0, jitter=0.02, seed=inputs.SEED_MIXTURE)
    proj = inputs.gen_projections(n, 16, inputs.SEED_PROJ)
    q = x.shape[0]
    log(f"image: {width}x{width} G-buffer, k={k}, generated in {time.time() - t0:.1f}s")
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    xd = d(x)
    m = ngd.Mixture(n, k)
    m.update(d(mix["mean"]), d(mix["factor"]), d(mix["weight"]), d(mix["colour"]))
    m.validate()
    rng = np.random.default_rng(inputs.SEED_QUERIES)
    idx = np.sort(rng.choice(q, sample, replace=False))
    t1 = time.perf_counter()
    fo = oracle.eval_mixture(mix["mean"], mix["factor"], mix["weight"], mix["colour"], x[idx])
    log(f"oracle on {sample} pixels: {time.perf_counter() - t1:.1f}s")

    def med(fn):
        out = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            out.append(a.elapsed_time(b))
        return float(np.median(out))

    f = torch.empty((q, 3), device="cuda")
    dense_ms = med(lambda: ngd.eval_mixture(m, None, xd, out=f))
    s3 = math.exp(-4.5)
    rows = []
    for tiling, tau in ((2, 1e-4), (0, 1e-4), (1, 1e-4), (2, s3), (0, s3)):
        p = ngd.default_params()
        p.tiling, p.tau = tiling, tau
        c = ngd.Cull().build(m, xd, proj, p)
        fc = ngd.eval_mixture(m, c, xd)
        torch.cuda.synchronize()
        st = c.stats()
        err = float(np.abs(fc[torch.from_numpy(idx).to("cuda")].double().cpu().numpy() - fo).max()
                    / max(np.abs(fo).max(), 1e-300))
        row = dict(tiling={0: "k-d", 1: "morton", 2: "image 16x16"}[tiling], tau=tau,
                   candidates=st["total"], fraction=st["total"] / max(st["ntiles"] * k, 1),
                   cull_ms=med(lambda: c.build(m, xd, proj, p)),
                   fwd_fp32_ms=med(lambda: ngd.eval_mixture(m, c, xd, out=f)),
                   fwd_bf16_ms=med(lambda: ngd.eval_mixture(m, c, xd, out=f,
                                                            precision=ngd.BF16_MFMA)),
                   err_fp32_vs_oracle=err)
        row["speedup_fwd_vs_dense"] = dense_ms / (row["cull_ms"] + row["fwd_fp32_ms"])
        log(f"image tiling={row['tiling']} tau={tau:.4g}: {row['fraction']:.4%} of pairs, cull "
            f"{row['cull_ms']:.3f} ms, fwd {row['fwd_fp32_ms']:.3f} / {row['fwd_bf16_ms']:.3f} ms, "
            f"err {err:.2e}")
        rows.append(row)

    # global conditioning: every input but the position constant over the image
    xc = np.array([0.0, 0.0, 1.0, 0.0, 0.0, 1.0, 0.5], np.float32)
    xg = inputs.gen_gbuffer(width, width, constant_features=xc)
    xgd = d(xg)
    xg3 = d(np.ascontiguousarray(xg[:, :3]))
    p10 = ngd.default_params()
    p10.tiling = 2
    c10 = ngd.Cull().build(m, xgd, proj, p10)
    f10 = ngd.eval_mixture(m, c10, xgd)
    proj3 = inputs.gen_projections(3, 16, inputs.SEED_PROJ)
    c3 = ngd.Cull()
    f3 = torch.empty((q, 3), device="cuda")
    w_src = d(mix["weight"])
    state = {}

    def cond_path():
        # the conditioned factor exp(-M_c/2) bounds every value of that
        # Gaussian on the image, so the ones below tau are dropped (the
        # threshold the 10-D cull applies per tile); the selection is done
        # in torch (one device-to-host read of the count)
        cm, cf, cw, cc = m.condition(3, xc)
        keep = torch.nonzero(cw > p10.tau * w_src).flatten()
        kk = int(keep.numel())
        if state.get("k") != kk:
            state["m3"], state["k"] = ngd.Mixture(3, kk), kk
        m3 = state["m3"]
        m3.update(cm[keep].contiguous(), cf[keep].contiguous(), cw[keep].contiguous(),
                  cc[keep].contiguous())
        c3.build(m3, xg3, proj3, p10)
        ngd.eval_mixture(m3, c3, xg3, out=f3)

    cond_path()
    torch.cuda.synchronize()
    state["m3"].validate()
    scale = float(f10.abs().max())
    diff = float((f10 - f3).abs().max()) / max(scale, 1e-300)
    fog = oracle.eval_mixture(mix["mean"], mix["factor"], mix["weight"], mix["colour"], xg[idx])
    err3 = float(np.abs(f3[torch.from_numpy(idx).to("cuda")].double().cpu().numpy() - fog).max()
                 / max(np.abs(fog).max(), 1e-300))
    glob = dict(xc=xc.tolist(), ms_10d=med(lambda: (c10.build(m, xgd, proj, p10),
                                                     ngd.eval_mixture(m, c10, xgd, out=f10))),
                ms_conditioned_3d=med(cond_path), candidates_10d=c10.stats()["total"],
                candidates_3d=c3.stats()["total"], k_conditioned_kept=state["k"],
                max_rel_diff_3d_vs_10d=diff,
                err_3d_vs_oracle=err3, value_scale=scale)
    log(f"global conditioning: 10-D cull+fwd {glob['ms_10d']:.3f} ms, condition+3-D cull+fwd "
        f"{glob['ms_conditioned_3d']:.3f} ms, rel diff {diff:.2e}, err vs oracle {err3:.2e}")
    print(json.dumps(dict(
        metric="cull on an image-coherent 10-D G-buffer: tilings and thresholds; global "
               "conditioning", unit="ms", n_gpus=1, data="synthetic", dtype="f32 / bf16+f32",
        config=dict(workload="10d-gbuffer", width=width, height=width, tile_pixels=16, n=n,
                    k=k, q=q, n_proj=16, error_sample=sample, reps=reps),
        dense_fp32_fwd_ms=dense_ms, rows=rows, global_conditioning=glob)), flush=True)


def _median_by_kernel(csv_path, counter=None):
    """Per kernel name: (dispatches, median value) of a rocprofv3 CSV -- the
    counter column of a --pmc run, or the duration of a --kernel-trace run."""
    import csv
    vals = {}
    for r in csv.DictReader(open(csv_path)):
        name = r["Kernel_Name"]
        if counter is not None:
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"])
        else:
            v = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
        vals.setdefault(name, []).append(v)
    return {k: (len(v), float(np.median(v))) for k, v in vals.items()}


def _short(name):
    """A kernel's name without namespace and argument list (mangled names
    demangled with c++filt)."""
    if name.startswith("_Z"):
        import re
        import subprocess
        try:
            out = subprocess.run(["c++filt", name], capture_output=True, text=True,
                                 check=True).stdout.strip()
        except (OSError, subprocess.CalledProcessError):
            out = name
        if out.startswith("_Z"):
            # names c++filt leaves mangled (bf16 vector arguments): the
            # kernel's name and its int / bool template arguments
            m = re.search(r"\d+(k_[A-Za-z0-9_]+?)I((?:L[ib]\d+E)+)E", name)
            if not m:
                return name
            args = re.findall(r"L([ib])(\d+)E", m.group(2))
            txt = [v if t == "i" else ("true" if v == "1" else "false") for t, v in args]
            return f"{m.group(1)}<{', '.join(txt)}>"
        name = out
    base = name.replace("void ", "", 1) if name.startswith("void ") else name
    base = base.replace("ngd::(anonymous namespace)::", "")
    depth = 0
    for i, ch in enumerate(base):
        depth += ch == "<"
        depth -= ch == ">"
        if ch == "(" and depth == 0:
            return base[:i]
    return base


def summarize_traffic(fetch_csv, write_csv, out_prefix):
    """HBM bytes per launch of each path's forward from two rocprofv3 --pmc
    runs of `bench.py --profile` (FETCH_SIZE, then WRITE_SIZE; KiB per
    dispatch), each scaled by what the counter reads for the run's closing
    device copy of 268,435,456 bytes.  Writes the JSON files the bench reads
    (with the forward sources' hash) and prints a markdown table."""
    fe = {(_short(k)): v for k, v in _median_by_kernel(fetch_csv, "FETCH_SIZE").items()}
    wr = {(_short(k)): v for k, v in _median_by_kernel(write_csv, "WRITE_SIZE").items()}
    copy = "__amd_rocclr_copyBuffer"
    # the calibration copy is the largest copy dispatch of the run
    import csv
    cf = max(float(r["Counter_Value"]) for r in csv.DictReader(open(fetch_csv))
             if r["Kernel_Name"].startswith(copy) and r["Counter_Name"] == "FETCH_SIZE")
    cw = max(float(r["Counter_Value"]) for r in csv.DictReader(open(write_csv))
             if r["Kernel_Name"].startswith(copy) and r["Counter_Name"] == "WRITE_SIZE")
    nbytes = 268435456
    ffac, wfac = nbytes / 1024 / cf, nbytes / 1024 / cw
    paths = dict(fp32=(["k_eval_items<10, true, false>", "k_eval_reduce"], (KERNEL_SRC,)),
                 bf16_mfma=(["k_mfma_filter<10, true, false>"], (MFMA_SRC, KERNEL_SRC)))
    lines = ["| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB |", "|---|---|---|---|"]
    for k in sorted(fe, key=lambda k: -fe[k][1]):
        if k in wr and fe[k][1] + wr[k][1] > 1024:
            lines.append(f"| `{k}` | {fe[k][0]} | {fe[k][1]:.0f} | {wr[k][1]:.0f} |")
    for name, (kerns, srcs) in paths.items():
        if not all(k in fe and k in wr for k in kerns):
            continue
        f_kib = sum(fe[k][1] for k in kerns)
        w_kib = sum(wr[k][1] for k in kerns)
        rec = dict(workload="10d-fwdbwd", path=name, kernels=kerns,
                   source_sha256_16=source_hash(*srcs),
                   sources=[os.path.relpath(x, ROOT) for x in srcs],
                   fetch_kib_per_launch_raw=f_kib, write_kib_per_launch_raw=w_kib,
                   copy_calibration=dict(bytes=nbytes, fetch_kib=cf, write_kib=cw,
                                         fetch_factor=ffac, write_factor=wfac),
                   hbm_bytes_per_launch=(f_kib * ffac + w_kib * wfac) * 1024)
        json.dump(rec, open(TRAFFIC_FILES[name], "w"), indent=1)
        lines.append(f"\n{name}: {rec['hbm_bytes_per_launch'] / 1e9:.3f} GB per forward "
                     f"(calibrated), source hash {rec['source_sha256_16']}")
    lines.append(f"\ncalibration copy of {nbytes} bytes: FETCH_SIZE {cf:.0f} KiB "
                 f"(factor {ffac:.3f}), WRITE_SIZE {cw:.0f} KiB (factor {wfac:.3f})")
    print("\n".join(lines))


def summarize_trace(stats_csv, top=40):
    """A markdown table of a rocprofv3 --kernel-trace --stats summary; with
    the per-dispatch trace beside it (`*_kernel_trace.csv`), a second table
    of each kernel's median over the main workload's dispatches: those of at
    least 0.4 times the kernel's longest, which leaves out the small
    hidden-target (K = 4,096) build and forward that the averages include."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    print("| kernel | calls | avg us | total ms | % |\n|---|---|---|---|---|")
    for r in rows[:top]:
        print(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
              f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |")
    trace_csv = stats_csv.replace("_kernel_stats.csv", "_kernel_trace.csv")
    if trace_csv == stats_csv or not os.path.exists(trace_csv):
        return
    dur = {}
    for r in csv.DictReader(open(trace_csv)):
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        dur.setdefault(_short(r["Kernel_Name"]), []).append(d)
    med = []
    for name, d in dur.items():
        big = [v for v in d if v >= 0.4 * max(d)]
        med.append((float(np.median(big)) * len(big), name, len(big), float(np.median(big))))
    med.sort(reverse=True)
    print("\nMain workload (dispatches of at least 0.4 x the kernel's longest):\n")
    print("| kernel | dispatches | median us |\n|---|---|---|")
    for _, name, n, m in med[:top]:
        print(f"| `{name}` | {n} | {m:.1f} |")


def summarize_counters(pmc_csv, kernel):
    """Median per dispatch of every counter a --pmc run collected for one
    kernel, and the matrix-core utilisation they give."""
    import csv
    vals = {}
    for r in csv.DictReader(open(pmc_csv)):
        if _short(r["Kernel_Name"]) == kernel:
            vals.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    med = {k: float(np.median(v)) for k, v in vals.items()}
    for k, v in sorted(med.items()):
        print(f"| {k} | {v:.4g} |")
    if "SQ_VALU_MFMA_BUSY_CYCLES" in med and "GRBM_GUI_ACTIVE" in med:
        # GRBM_GUI_ACTIVE summed over the 8 XCDs; 1,024 SIMDs
        util = med["SQ_VALU_MFMA_BUSY_CYCLES"] / (med["GRBM_GUI_ACTIVE"] / 8 * 1024)
        print(f"\nMFMA busy: {util:.3f} of the SIMD cycles the kernel spans")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="10d-fwdbwd")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="time only --workload, not the other configurations")
    ap.add_argument("--precision", default="both", choices=["fp32", "bf16_mfma", "both"],
                    help="forward arithmetic of the timed step; 'both' times the step once "
                         "with each and reports the faster as the headline")
    ap.add_argument("--profile", action="store_true",
                    help="short run for rocprofv3 (3 steps, 1 warmup, no CPU/dense legs, "
                         "no other configurations) plus one 256 MiB device copy to "
                         "calibrate memory counters")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the step benchmark, sweep the cull threshold tau and "
                         "the tile size and print one line of rows")
    ap.add_argument("--image", action="store_true",
                    help="instead of the step benchmark, the cull on an image-coherent "
                         "G-buffer (16 x 16 pixel tiles against the k-d and Morton orders) "
                         "and the global-conditioning case; prints its own line")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter CSVs of `--profile` runs into the "
                         "traffic files under profiles/ and print a table; no GPU")
    ap.add_argument("--summarize-trace", metavar="KERNEL_STATS_CSV",
                    help="print a rocprofv3 --kernel-trace --stats summary as a table; no GPU")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("PMC_CSV", "KERNEL"),
                    help="print one kernel's counters from a rocprofv3 --pmc CSV; no GPU")
    ap.add_argument("--fit", type=int, default=0, metavar="STEPS",
                    help="instead of the step benchmark, run the 10-D fitting loop for "
                         "STEPS steps and print its own line (ms/step, losses, K)")
    ap.add_argument("--fit-lr", type=float, default=2e-3,
                    help="Adam learning rate of the means, factors and colours in --fit")
    ap.add_argument("--fit-lr-child", type=float, default=1e-2,
                    help="Adam learning rate of the children's relative parameters in --fit")
    ap.add_argument("--fit-lr-alpha", type=float, default=5e-2,
                    help="Adam learning rate of the log-brightnesses in --fit")
    ap.add_argument("--fit-init-scale", type=float, default=0.7,
                    help="factor scale of the start relative to the target's in --fit")
    ap.add_argument("--fit-child-alpha", type=float, default=1e-3,
                    help="brightness of a new child in --fit")
    ap.add_argument("--fit-child-jitter", type=float, default=0.3,
                    help="spread of a new child's relative parameters in --fit")
    ap.add_argument("--fit-target", default="coarse", choices=["coarse", "detail"],
                    help="hidden target of --fit: the K=4,096 mixture, or the same with "
                         "narrower components in place of each (--fit-detail-*)")
    ap.add_argument("--fit-per-component", type=float, default=8,
                    help="Gaussians of the --fit start per target component (below 1: one "
                         "on that fraction of the components)")
    ap.add_argument("--fit-detail-sub", type=int, default=16,
                    help="components in place of each coarse one for --fit-target detail")
    ap.add_argument("--fit-detail-narrow", type=float, default=0.35,
                    help="their factor scale relative to the coarse one's")
    ap.add_argument("--fit-adam-eps", type=float, default=1e-15,
                    help="Adam's epsilon in --fit")
    ap.add_argument("--fit-checkpoint", default=None,
                    help="file the fit's final state is saved to (--fit)")
    args = ap.parse_args()
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic, None)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    if args.profile:
        args.steps, args.warmup = 3, 1
        args.no_cpu_baseline = args.no_dense = args.no_configs = True
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2405_20067_amd import ngd
    torch.cuda.set_device(0)
    ngd.lib()
    if args.fit > 0:
        fit_bench(args.fit, "fp32" if args.precision == "fp32" else "bf16_mfma",
                  lr=args.fit_lr, lr_alpha=args.fit_lr_alpha, lr_child=args.fit_lr_child,
                  init_scale=args.fit_init_scale, per_component=args.fit_per_component,
                  child_alpha=args.fit_child_alpha, child_jitter=args.fit_child_jitter,
                  checkpoint=args.fit_checkpoint, target_kind=args.fit_target,
                  detail_sub=args.fit_detail_sub, detail_narrow=args.fit_detail_narrow,
                  adam_eps=args.fit_adam_eps)
        return
    if args.sweep:
        sweep_bench()
        return
    if args.image:
        image_bench()
        return
    precisions = ["fp32", "bf16_mfma"] if args.precision == "both" else [args.precision]
    rec, (w, mix, x) = run_workload(args.workload, args, precisions, not args.no_dense,
                                    args.steps, args.warmup, profile_copy=args.profile)
    torch.cuda.empty_cache()
    others = {}
    if not args.no_configs:
        for name in OTHER_WORKLOADS:
            if name == args.workload:
                continue
            others[name], _ = run_workload(name, args, precisions, not args.no_dense,
                                           max(3, args.steps // 2), max(1, args.warmup))
            torch.cuda.empty_cache()

    cpu = cpu1 = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle (all threads, then one) ...")
        cpu = cpu_baseline(w, mix, x, args.cpu_seconds)
        cpu1 = cpu_baseline(w, mix, x, max(2.0, args.cpu_seconds / 3), threads=1)
        cpu["single_core"] = cpu1

    head = rec["head"]
    out = dict(
        metric="Gaussian-query evals/sec, culled fwd+bwd 10-D, + % HBM/MFMA roofline",
        value=rec["value"], unit="Gaussian-query evals/s (dense-equivalent Q*K per step time)",
        n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=rec["ms_per_step"],
        higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f32" if head == "fp32" else "bf16+f32",
        data="synthetic",
        config=dict(workload=rec["workload"], description=rec["description"], n=rec["n"],
                    k=rec["k"], q=rec["q"], k_target=rec["k_target"],
                    near_frac=rec["near_frac"], n_proj=rec["n_proj"], tau=rec["tau"],
                    tile=rec["tile"], tiling=rec["tiling"]),
        precision=head, stages_ms=rec["stages_ms"], paths=rec["paths"], cull=rec["cull"],
        candidate_pairs_per_s_forward=rec["candidate_pairs_per_s_forward"],
        dense_fp32=rec["dense_fp32"], roofline=rec["paths"][head]["roofline"],
        cpu_baseline=cpu, configs=others)
    if cpu is not None:
        out["speedup_vs_cpu_oracle"] = rec["value"] / cpu["value"]
        out["speedup_vs_cpu_oracle_1core"] = rec["value"] / cpu1["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
