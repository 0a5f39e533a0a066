"""Benchmark: split-and-merge dictionary learning with plain and learned-proposal OMP on one
MI355X, at 8x8-patch scale (m=64, K=256, s=8).

One step = one pass of the whole hot path over one synthetic batch, inputs resident in HBM:
  1. Algorithm 1 on N=100000 signals: 20 subsets of 5000, local K=256, s=8, 20 MOD
     iterations each (all subsets batched per launch, iterations replayed as a HIP graph);
     merge of the 5120 pooled atoms to K=256 with s=4 and 20 iterations; final OMP coding of
     all N signals at s=8;
  2. labels for the proposer: plain OMP of 200000 fresh training signals with the learned D;
  3. proposer training (MLP 64-512-512-256, BF16 GEMMs, Adam) for `--epochs` epochs;
  4. coding of 100000 fresh evaluation signals, plain and with the trained proposer (top 24
     candidates, full-OMP fallback when ||r|| > 1.1 x the RMS plain residual of the training
     pairs).
After the timed steps the fallback threshold is swept (1.1 x down to 0.8 x) to report learned
vs plain throughput at equal representation RMSE (ratio within 1 %).
value = signals sparse-coded at (m=64, K=256, s=8) per second of the whole step (the local
codings of every iteration, the final coding, the labels and both evaluation codings).

Prints one JSON line (rank 0, single GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

ALGO_FLOPS_NOTE = ("2mK (correlations) + K s(s-1) (correlation updates) + sum_k [(k-1)^2 + 2k^2] "
                   "(Cholesky rows and coefficients) flops per signal (m=64,K=256,s=8: 47652); the s K "
                   "argmax compares are counted apart as ALU operations")

FP32_PEAK = 157.3          # TFLOP/s, MI355X dense FP32 (matrix cores; vector with packed FP32)
FP32_VALU_UNPACKED = 78.6  # TFLOP/s, MI355X FP32 vector issue without packed FP32 instructions


def omp_flops_per_signal(m: int, K: int, s: int) -> int:
    """Algorithmic FP32 flops of one OMP coding: the correlations D^T y, the correlation
    updates of the greedy steps and the Cholesky data and coefficients."""
    return 2 * m * K + K * s * (s - 1) + sum((k - 1) ** 2 + 2 * k * k for k in range(1, s + 1))


def omp_alu_ops_per_signal(K: int, s: int) -> int:
    """The argmax compares of the greedy steps (s passes over K correlations)."""
    return s * K


FP16_MFMA_PEAK = 2500.0    # TFLOP/s, MI355X dense FP16 matrix cores


def omp_mix_ceiling(m: int, K: int, s: int) -> float:
    """The ceiling this build's flop mix faces: the correlations on the FP16 matrix cores, three
    products per FP32 product (the hi/lo split) at 2.5 PFLOP/s, the rest on the vector ALUs, which
    issue at most 78.6 TFLOP/s without packed FP32 instructions (this build does not emit them):
    the harmonic combination, in algorithmic FP32 flops per second."""
    f = omp_flops_per_signal(m, K, s)
    a0 = 2 * m * K
    return f / (3 * a0 / FP16_MFMA_PEAK + (f - a0) / FP32_VALU_UNPACKED)


def omp_bytes_per_signal(m: int, s: int) -> int:
    """Algorithmic HBM bytes of one OMP coding: the signal in, the ELL code out."""
    return 4 * m + 8 * s + 4


def measured_traffic(kernel: str):
    """HBM bytes per launch of the plain OMP pass by this kernel instantiation, from the
    committed rocprofv3 PMC summary; None when that instantiation was not measured or the kernel
    source has changed since the counters were taken."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "omp_fused_traffic.json")) as f:
            rec = json.load(f)
        with open(os.path.join(ROOT, "paper_1403_4781_amd", "csrc", "omp_kernel.h"), "rb") as f:
            sha = hashlib.sha1(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("omp_kernel_sha1") != sha:
        return None
    return rec.get("bytes_per_launch", {}).get(kernel)


def train_roofline(widths, samples: int, ms: float):
    """The proposer training phase (the largest share of the step) against the dense BF16 MFMA
    peak: forward, hidden deltas and weight gradients are 3 x 2 x sum(w_l w_{l+1}) flops per
    sample (the first layer's input delta is not formed: 2 x w_0 w_1 less), timed over the whole
    phase (every launch, the Adam updates and the per-epoch host shuffles included)."""
    pairs = sum(a * b for a, b in zip(widths[:-1], widths[1:]))
    f = 6 * pairs - 2 * widths[0] * widths[1]
    achieved = f * samples / (ms * 1e-3) / 1e12
    return {"phase": "proposer training (fused network kernel + weight gradients with Adam, per batch)",
            "bound": "mfma", "achieved": achieved, "peak": 2500.0, "unit": "TFLOP/s", "frac": achieved / 2500.0,
            "per_sample_flops": f, "samples": samples, "ms": ms}


def omp_kernel_name(h, m: int, K: int, s: int) -> str:
    """The fused OMP instantiation the handle runs for (m, K, s): lanes per signal G, entries per
    lane EM = Kpad / G, steps SM (the smallest instantiated >= s: 8 for s <= 8), 16 TT signals per
    item."""
    lanes, spi = h.get_tile(m, K, s)
    kpad = (K + 63) // 64 * 64
    sm = 8 if s <= 8 else (12 if s <= 12 else 16)
    return f"omp_fused<{kpad // lanes}, {sm}, {lanes}, {spi // 16}>"


def cpu_baseline(w, sample_subsets: int, sample_n: int, iters: int, one_thread_subsets: int = 1):
    """The FP64 oracle on a bounded sample of the same workload, timed on the host cores: on all
    of them, and on one thread over a smaller sample."""
    import oracle
    oracle.build()

    def run(L):
        idx = w.perm[: L * sample_n]
        Ys = w.Y[idx]
        perm = np.arange(len(idx), dtype=np.int64)
        offs = np.arange(L + 1, dtype=np.int64) * sample_n
        t0 = time.perf_counter()
        oracle.split_merge(Ys, perm, offs, [256] * L, [8] * L, 256, iters, iters, 4, 8)
        dt = time.perf_counter() - t0
        return L * sample_n * (iters + 1) + len(idx), dt

    codings, dt = run(sample_subsets)
    threads = oracle.threads()
    oracle.set_threads(1)
    try:
        c1, dt1 = run(one_thread_subsets)
    finally:
        oracle.set_threads(threads)
    return {"value": codings / dt, "unit": "signals sparse-coded/sec (m=64,K=256,s=8)", "cores": threads,
            "kind": "oracle",
            "sample": f"Algorithm 1 on {sample_subsets} subsets x {sample_n} signals of the same data, "
                      f"{iters}+{iters} iterations, final coding of {sample_subsets * sample_n}: {codings} codings "
                      f"in {dt:.2f} s",
            "value_1thread": c1 / dt1,
            "sample_1thread": f"the same on {one_thread_subsets} subset(s) x {sample_n} signals: {c1} codings in "
                              f"{dt1:.2f} s on one thread"}


def run_batched(args, smdl, synth, torch, dev):
    """The uneven split phase: 64 subsets of 1000-20000 signals, local K in {64, 128, 192, 256}, s in
    {4, 8, 12}, 20 iterations, then the merge and the final coding, once with every stage of all
    subsets in one launch (each iteration a replayed HIP graph) and once with per-subset launches."""
    w = synth.batched_split(iters=args.iters)
    Y = torch.from_numpy(w.Y).to(dev)
    perm = torch.from_numpy(w.perm).to(dev)
    h = smdl.Handle(0)
    res = {}
    for name, flags in (("batched", 0), ("per_subset", smdl.SMDL_PER_SUBSET_LAUNCH)):
        for _ in range(args.warmup):
            h.split_merge_learn(Y, perm, w.offsets, w.K_local, w.s_local, w.K, w.iters_local, w.iters_merge,
                                w.s_merge, w.s_final, flags=flags)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ph = []
        for _ in range(args.steps):
            h.split_merge_learn(Y, perm, w.offsets, w.K_local, w.s_local, w.K, w.iters_local, w.iters_merge,
                                w.s_merge, w.s_final, flags=flags)
            ph.append(h.phase_ms())
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        local_ms = float(np.mean([p[0] for p in ph]))
        res[name] = {"ms_per_run": dt * 1e3, "local_ms": local_ms, "merge_ms": float(np.mean([p[1] for p in ph])),
                     "final_ms": float(np.mean([p[2] for p in ph])),
                     "local_signals_coded_per_s": w.N * (w.iters_local + 1) / (local_ms * 1e-3)}
    flops = sum(int(n) * omp_flops_per_signal(64, int(k), int(s_))
                for n, k, s_ in zip(np.diff(w.offsets), w.K_local, w.s_local))
    out = {"metric": "signals sparse-coded/sec in the split phase (batched uneven subsets)",
           "value": res["batched"]["local_signals_coded_per_s"], "unit": "signals/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
           "config": {"workload": w.name, "N": w.N, "L": w.L, "K_local": "64/128/192/256", "s_local": "4/8/12",
                      "iters_local": w.iters_local, "iters_merge": w.iters_merge},
           "batched": res["batched"], "per_subset": res["per_subset"],
           "batched_speedup_local": res["per_subset"]["local_ms"] / res["batched"]["local_ms"],
           "omp_flops_per_pass": flops,
           "omp_tflops_local": flops * (w.iters_local + 1) / (res["batched"]["local_ms"] * 1e-3) / 1e12}
    print(json.dumps(out), flush=True)


def run_large(args, smdl, synth, torch, dev):
    """The large workload: m=256, N=1e6 in 100 uneven subsets, local K=512 s=16 (20 iterations), merge
    to K=1024 (s=8), final s=16 coding of all N; then the 256-1024-1024-1024 proposer trained on
    200000 labelled pairs and plain vs proposed coding (48 candidates) of 100000 fresh signals."""
    w = synth.large_scale(iters=args.iters)
    Ytr = synth.fresh_signals(w, synth.STREAM_TRAIN, 200000, 16, 0.02)
    Yev = synth.fresh_signals(w, synth.STREAM_EVAL, 100000, 16, 0.02)
    print(f"# large workload drawn: N={w.N}, m={w.m}", file=sys.stderr, flush=True)
    Y = torch.from_numpy(w.Y).to(dev)
    perm = torch.from_numpy(w.perm).to(dev)
    Yt = torch.from_numpy(Ytr).to(dev)
    Ye = torch.from_numpy(Yev).to(dev)
    h = smdl.Handle(0)
    widths = [256, 1024, 1024, 1024]
    Ws, bs = synth.mlp_init(widths)
    if args.train_only:
        D = torch.from_numpy(synth.gaussian_dictionary(np.random.default_rng(1), w.m, w.K).astype(np.float32)).to(dev)
        labels = h.omp_code(D, Yt, 16)
        prop = h.proposer(Ws, bs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses = prop.train(Yt, labels, epochs=args.train_only, batch=1024, lr=1e-3, shuffle_seed=1)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        prop.close()
        print(json.dumps({"train_only": args.train_only, "widths": widths, "ms": ms,
                          "steps": args.train_only * (Ytr.shape[0] // 1024), "losses": losses}))
        return

    def step():
        info = {}
        D, X, _, _ = h.split_merge_learn(Y, perm, w.offsets, w.K_local, w.s_local, w.K, w.iters_local,
                                         w.iters_merge, w.s_merge, w.s_final)
        info["phase_ms"] = h.phase_ms()
        labels, rn_tr = h.omp_code(D, Yt, 16, res_norm=True)
        rms_tr = float(torch.sqrt((rn_tr.double() ** 2).mean()).item())
        prop = h.proposer(Ws, bs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prop.train(Yt, labels, epochs=args.epochs, batch=1024, lr=1e-3, shuffle_seed=1)
        torch.cuda.synchronize()
        info["train_ms"] = (time.perf_counter() - t0) * 1e3
        Xp = h.omp_code(D, Ye, 16)
        info["plain_kernel_ms"] = h.last_kernel_ms()
        Xl, _, nfb, _ = h.omp_code_proposed(prop, D, Ye, 16, 48, 1.1 * rms_tr)
        torch.cuda.synchronize()
        info.update(prop_ms=h.prop_phase_ms(), nfb=nfb, D=D, Xp=Xp, Xl=Xl, prop=prop, rms_tr=rms_tr)
        return info

    for _ in range(args.warmup):
        step()["prop"].close()
        print("# warmup step done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        infos.append(step())
        if len(infos) > 1:
            infos[-2]["prop"].close()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    last = infos[-1]
    D = last["D"]

    def rmse(X):
        Xd = X.dense(1024).double()
        R = Ye.double() - Xd @ D.double()
        return float(torch.sqrt((R ** 2).mean()).item())
    r_plain, r_learn = rmse(last["Xp"]), rmse(last["Xl"])
    curve = []
    for mult in (1.1, 1.0, 0.9, 0.8):
        Xm, _, nfm, _ = h.omp_code_proposed(last["prop"], D, Ye, 16, 48, mult * last["rms_tr"])
        torch.cuda.synchronize()
        curve.append({"eps_mult": mult, "rmse_ratio": rmse(Xm) / r_plain, "fallback_rate": nfm / Yev.shape[0],
                      "learned_signals_per_s": Yev.shape[0] / (sum(h.prop_phase_ms()) * 1e-3)})
    last["prop"].close()
    kms = float(np.mean([i["plain_kernel_ms"] for i in infos]))
    plain_sps = Yev.shape[0] / (kms * 1e-3)
    learned_sps = Yev.shape[0] / (sum(last["prop_ms"]) * 1e-3)
    codings = w.N * (w.iters_local + 1) + w.N + Ytr.shape[0] + 2 * Yev.shape[0]
    f_final = omp_flops_per_signal(256, 1024, 16)
    out = {"metric": "signals sparse-coded/sec (m=256,K=1024,s=16), learned vs plain",
           "value": codings / dt, "unit": "signals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": dt * 1e3, "higher_is_better": True,
           "config": {"workload": w.name + " + proposer_256-1024-1024-1024_top48", "N": w.N, "L": w.L,
                      "K_local": 512, "s_local": 16, "K": 1024, "s_merge": 8, "s_final": 16,
                      "iters_local": w.iters_local, "iters_merge": w.iters_merge, "train_pairs": int(Ytr.shape[0]),
                      "eval_signals": int(Yev.shape[0]), "epochs": args.epochs, "codings_per_step": codings},
           "phase_ms": {"local": last["phase_ms"][0], "merge": last["phase_ms"][1], "final": last["phase_ms"][2],
                        "proposer_train": float(np.mean([i["train_ms"] for i in infos])),
                        "plain_eval_kernel": kms, "proposer_net_topk": last["prop_ms"][0],
                        "proposer_restricted": last["prop_ms"][1], "proposer_fallback": last["prop_ms"][2]},
           "plain_signals_per_s": plain_sps, "learned_signals_per_s": learned_sps,
           "learned_vs_plain": learned_sps / plain_sps, "rmse_ratio": r_learn / r_plain,
           "fallback_rate": last["nfb"] / Yev.shape[0], "learned_vs_plain_curve": curve,
           "plain_final_roofline": {"bound": "alu", "per_signal_flops": f_final,
                                    "alu_ops_per_signal": omp_alu_ops_per_signal(1024, 16),
                                    "achieved": f_final * Yev.shape[0] / (kms * 1e-3) / 1e12, "peak": FP32_PEAK,
                                    "unit": "TFLOP/s",
                                    "frac": f_final * Yev.shape[0] / (kms * 1e-3) / 1e12 / FP32_PEAK,
                                    "mix_ceiling": omp_mix_ceiling(256, 1024, 16)}}
    print(json.dumps(out), flush=True)


def run_e1(args, smdl, synth, torch, dev):
    """The paper's synthetic experiment (Section 3.1, Table 1) through the library: the standard
    alternation (K = 60, s = 6) against split-and-merge (40 x 1000, K_1 = 50, s_1 = 3, merged to
    K = 60 at s_2 = 2, final coding at s = 6) on noise-free signals of a 30 x 60 Gaussian
    dictionary, averaged over independent trials; the FP64 oracle runs the first trials on the
    same inputs and is timed beside the GPU."""
    from paper_1403_4781_amd import evaluate
    h = smdl.Handle(0)
    rows = {"standard": [], "split_merge": [], "split_merge_composed": []}
    for t in range(args.trials):
        w = synth.synthetic_e1(t, iters=args.e1_iters)
        Y = torch.from_numpy(w.Y).to(dev)
        perm = torch.from_numpy(w.perm).to(dev)
        for name in rows:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name == "standard":
                D, X = h.learn(Y, w.K, 6, args.e1_iters)
            else:
                # the composed form (Proposition 1) replaces the final coding by X = Z X1
                flags = smdl.SMDL_COMPOSE_CODES if name == "split_merge_composed" else 0
                D, X, _, _ = h.split_merge_learn(Y, perm, w.offsets, w.K_local, w.s_local, w.K, w.iters_local,
                                                 w.iters_merge, w.s_merge, w.s_final, flags=flags)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            Dn = D.cpu().numpy()
            idx, coef, nnz = (a.cpu().numpy() for a in (X.idx, X.coef, X.nnz))
            rows[name].append({"mse_db": evaluate.mse_db(w.Y, Dn, idx, coef, nnz),
                               "recovery": evaluate.atom_recovery(w.D0, Dn), "s": sec,
                               "mean_nnz": float(nnz.mean())})
    ora = {"standard": [], "split_merge": []}
    if args.e1_oracle_trials > 0:
        import oracle
        oracle.build()
        for t in range(min(args.e1_oracle_trials, args.trials)):
            w = synth.synthetic_e1(t, iters=args.e1_iters)
            for name in ("standard", "split_merge"):
                t0 = time.perf_counter()
                if name == "standard":
                    D, X = oracle.learn(w.Y, w.K, 6, args.e1_iters)
                else:
                    D, X, _, _ = oracle.split_merge(w.Y, w.perm, w.offsets, w.K_local, w.s_local, w.K,
                                                    w.iters_local, w.iters_merge, w.s_merge, w.s_final)
                sec = time.perf_counter() - t0
                ora[name].append({"mse_db": evaluate.mse_db(w.Y, D, X.idx, X.coef, X.nnz),
                                  "recovery": evaluate.atom_recovery(w.D0, D), "s": sec})

    def summary(r):
        if not r:
            return None
        return {"mse_db_mean": float(np.mean([x["mse_db"] for x in r])),
                "mse_db_std": float(np.std([x["mse_db"] for x in r])),
                "recovery_pct_mean": 100.0 * float(np.mean([x["recovery"] for x in r])),
                "recovery_pct_std": 100.0 * float(np.std([x["recovery"] for x in r])),
                "seconds_per_trial": float(np.mean([x["s"] for x in r])), "trials": len(r),
                "mean_nnz": float(np.mean([x.get("mean_nnz", 0.0) for x in r])), "per_trial": r}
    out = {"metric": "E1: training MSE (dB) and atom recovery (%), standard vs split-and-merge",
           "config": {"workload": "synthetic_e1 (m=30, K=60, N=40000, s=6, noise-free)", "L": 40, "K_local": 50,
                      "s_local": 3, "s_merge": 2, "s_final": 6, "iters": args.e1_iters, "trials": args.trials},
           "gpu": {k: summary(v) for k, v in rows.items()},
           "oracle": {k: summary(v) for k, v in ora.items()},
           "oracle_threads": None,
           "paper_table1": {"standard": {"mse_db": -21.18, "recovery_pct": 94.27, "seconds": 158.16},
                            "split_merge": {"mse_db": -15.91, "recovery_pct": 85.53, "seconds": 5.95},
                            "note": "20 trials; the paper states neither its iteration count nor its hardware"}}
    if args.e1_oracle_trials > 0:
        import oracle
        out["oracle_threads"] = oracle.threads()
    print(json.dumps(out), flush=True)


def run_denoise(args, smdl, synth, torch, dev):
    """The image-denoising experiment of Section 3.2 on synthetic images (the paper's images are
    not available): dictionaries learned from 10^5 clean 8 x 8 patches, both started from the
    overcomplete DCT and run 100 iterations (standard: K = 256 at s = 8; split-and-merge: 20 x 5000,
    local K = 128 at s = 8, merged to K = 256 at s = 4); then every patch of three test images with
    white Gaussian noise of sigma in {10, 15, 20, 25, 50} (5 realizations) is coded with
    eps = 8.5 sigma (at most 16 atoms) and the overlapping estimates are averaged."""
    from paper_1403_4781_amd import evaluate
    g = synth.rng_streams(synth.SEED_BASE + 200)
    train_imgs = [synth.synthetic_image(g[0], 256, 256) for _ in range(8)]
    Yp = synth.image_patches(g[1], train_imgs, 100000, 8)
    Y = torch.from_numpy(Yp).to(dev)
    h = smdl.Handle(0)
    D256 = torch.from_numpy(synth.odct(8, 16, 16).astype(np.float32)).to(dev)
    D128 = torch.from_numpy(synth.odct(8, 16, 8).astype(np.float32)).to(dev)
    perm = torch.from_numpy(g[2].permutation(100000).astype(np.int64)).to(dev)
    offs = np.arange(21, dtype=np.int64) * 5000
    it = args.e1_iters
    dicts, train_s = {}, {}
    for name in ("standard", "split_merge"):
        h.learn(Y, 256, 8, 1, codes=False, D_init=D256)          # warm-up of every shape
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if name == "standard":
            D, _ = h.learn(Y, 256, 8, it, codes=False, D_init=D256)
        else:
            D, _, _, _ = h.split_merge_learn(Y, perm, offs, np.full(20, 128, np.int32), np.full(20, 8, np.int32), 256,
                                             it, it, 4, 8, codes=False, D_local_init=D128, D_merge_init=D256)
        torch.cuda.synchronize()
        train_s[name] = time.perf_counter() - t0
        dicts[name] = D
    test_imgs = [synth.synthetic_image(g[3], 256, 256) for _ in range(3)]
    rows = []
    den_s = []
    for sigma in (10.0, 15.0, 20.0, 25.0, 50.0):
        rng = np.random.default_rng(int(sigma))
        r = {"sigma": sigma, "psnr_in": [], "standard": [], "split_merge": []}
        for im in test_imgs:
            for _ in range(5):
                noisy = (im + sigma * rng.standard_normal(im.shape)).astype(np.float32)
                nt = torch.from_numpy(noisy).to(dev)
                r["psnr_in"].append(evaluate.psnr(im, noisy))
                for name in ("standard", "split_merge"):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    out = h.denoise(nt, dicts[name], 8, 8.5 * sigma, 16)
                    torch.cuda.synchronize()
                    den_s.append(time.perf_counter() - t0)
                    r[name].append(evaluate.psnr(im, out.cpu().numpy()))
        rows.append({k: (float(np.mean(v)) if isinstance(v, list) else v) for k, v in r.items()})
    patches = 249 * 249
    out = {"metric": "denoising PSNR (dB), standard vs split-and-merge dictionaries; training seconds",
           "config": {"workload": "synthetic images 256 x 256, 8 x 8 patches, 1e5 training patches",
                      "iters": it, "K": 256, "s": 8, "L": 20, "K_local": 128, "s_merge": 4, "eps": "8.5 sigma",
                      "s_max": 16, "test_images": 3, "realizations": 5},
           "train_seconds": train_s, "psnr": rows,
           "denoise_ms_per_image": 1e3 * float(np.median(den_s)),
           "denoise_patches_per_s": patches / float(np.median(den_s))}
    if args.e1_oracle_trials > 0:
        import oracle
        oracle.build()
        im = test_imgs[0]
        noisy = (im + 20.0 * np.random.default_rng(20).standard_normal(im.shape)).astype(np.float32)
        t0 = time.perf_counter()
        ref, _ = oracle.denoise(noisy, dicts["standard"].cpu().numpy(), 8, 8.5 * 20.0, 16)
        sec = time.perf_counter() - t0
        gpu = h.denoise(torch.from_numpy(noisy).to(dev), dicts["standard"], 8, 8.5 * 20.0, 16).cpu().numpy()
        out["oracle"] = {"seconds_per_image": sec, "threads": oracle.threads(),
                         "psnr_oracle": evaluate.psnr(im, ref), "psnr_gpu": evaluate.psnr(im, gpu),
                         "psnr_gpu_vs_oracle": evaluate.psnr(ref, gpu)}
    out["paper_context"] = ("Tables 2-3: standard images and IISc building images (not available); "
                            "training 1.25e3 s vs 33.59 s; the split-and-merge dictionary within 0.1-0.3 dB")
    print(json.dumps(out), flush=True)


def run_modsolve(args, smdl, synth, torch, dev):
    """The MOD update at the shapes of the workloads, with each factorisation of the normal
    equations forced in turn (2: one work group per dictionary, 1: multi-work-group panels), then
    in the fixed-order mode: one JSON line per shape with the wall time of one smdl_mod_update
    (transpose, products, solve, normalisation; mean of 10 after one warm-up) and the largest
    differences of the results."""
    h = smdl.Handle(0)
    rng = np.random.default_rng(synth.SEED_BASE + 300)
    shapes = [("merge, patch scale", 64, 256, 4, 5120), ("local, patch scale", 64, 256, 8, 5000),
              ("local, large", 256, 512, 16, 10000), ("merge, large", 256, 1024, 8, 51200),
              ("synthetic experiment", 30, 64, 6, 1000)]
    for name, m, K, s, N in shapes:
        idx = torch.rand(N, K, device=dev).argsort(dim=1)[:, :s].int().contiguous()
        X = smdl.Codes(idx, torch.randn(N, s, device=dev), torch.full((N,), s, dtype=torch.int32, device=dev))
        Y = torch.randn(N, m, device=dev)
        D0 = torch.from_numpy(synth.gaussian_dictionary(rng, m, K).astype(np.float32)).to(dev)
        res = {}
        # (factorisation, handle flags): each forced factorisation, then the default one in the
        # fixed-order mode (code lists and product sums in a fixed order)
        for key, solver, flags in ((2, 2, 0), (1, 1, 0), ("fixed", 0, smdl.SMDL_DETERMINISTIC)):
            h.set_mod_solver(solver)
            h.set_flags(flags)
            D = D0.clone()
            h.mod_update(Y, X, D)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(10):
                D = D0.clone()
                h.mod_update(Y, X, D)
            torch.cuda.synchronize()
            res[key] = ((time.perf_counter() - t0) / 10 * 1e3, D.cpu().numpy())
        h.set_mod_solver(0)
        h.set_flags(0)
        print(json.dumps({"shape": name, "m": m, "K": K, "s": s, "N": N,
                          "one_work_group_ms": round(res[2][0], 3), "multi_work_group_ms": round(res[1][0], 3),
                          "max_abs_difference": float(np.abs(res[1][1] - res[2][1]).max()),
                          "fixed_order_ms": round(res["fixed"][0], 3),
                          "fixed_order_max_abs_difference": float(np.abs(res["fixed"][1] - res[1][1]).max())}),
              flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-subsets", type=int, default=20)
    ap.add_argument("--cpu-n", type=int, default=5000)
    ap.add_argument("--cpu-iters", type=int, default=20)
    ap.add_argument("--omp-only", type=int, default=0,
                    help="only run the plain OMP coding of the 100000 signals this many times (for profilers)")
    ap.add_argument("--omp-tile", default="",
                    help="with --omp-only: 'lanes,signals_per_item' to force that OMP tile")
    ap.add_argument("--train-only", type=int, default=0,
                    help="only train the proposer this many epochs on the 200000 training pairs (for profilers; "
                         "the default and the large configuration)")
    ap.add_argument("--trials", type=int, default=20, help="e1: independent trials")
    ap.add_argument("--e1-iters", type=int, default=100, help="e1: iterations of every learning stage")
    ap.add_argument("--e1-oracle-trials", type=int, default=1, help="e1: trials also run by the FP64 oracle")
    ap.add_argument("--config", default="split_merge", choices=["split_merge", "batched", "large", "e1", "denoise", "modsolve"],
                    help="batched: the 64-subset uneven split phase, batched vs per-subset launches; "
                         "large: m=256, K=1024, N=1e6 with the 256-1024-1024-1024 proposer (one JSON line each); "
                         "modsolve: the MOD update with each factorisation forced (one JSON line per shape)")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="only run a plain device copy of this many MiB three times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_1403_4781_amd as smdl
    from paper_1403_4781_amd import synth

    dev = torch.device("cuda:0")
    if args.config == "batched":
        run_batched(args, smdl, synth, torch, dev)
        return
    if args.config == "large":
        run_large(args, smdl, synth, torch, dev)
        return
    if args.config == "e1":
        run_e1(args, smdl, synth, torch, dev)
        return
    if args.config == "denoise":
        run_denoise(args, smdl, synth, torch, dev)
        return
    if args.config == "modsolve":
        run_modsolve(args, smdl, synth, torch, dev)
        return
    if args.copy_calib:
        n = args.copy_calib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_mib": args.copy_calib, "bytes_read_per_copy": 4 * n,
                          "bytes_written_per_copy": 4 * n}))
        return
    w = synth.patch_scale(N=100000, L=20, iters=args.iters)
    Ytr = synth.fresh_signals(w, synth.STREAM_TRAIN, 200000, 8, 0.02)
    Yev = synth.fresh_signals(w, synth.STREAM_EVAL, 100000, 8, 0.02)
    h = smdl.Handle(0)
    Y = torch.from_numpy(w.Y).to(dev)
    Yt = torch.from_numpy(Ytr).to(dev)
    Ye = torch.from_numpy(Yev).to(dev)
    perm = torch.from_numpy(w.perm).to(dev)
    widths = [64, 512, 512, 256]
    Ws, bs = synth.mlp_init(widths)
    torch.cuda.synchronize()

    if args.omp_only:
        D = torch.from_numpy(synth.gaussian_dictionary(np.random.default_rng(1), 64, 256).astype(np.float32)).to(dev)
        if args.omp_tile:
            lanes, spi = (int(x) for x in args.omp_tile.split(","))
            h.set_autotune(False)
            h.set_tile(256, 8, lanes, spi)
        for _ in range(args.omp_only):
            h.omp_code(D, Y, 8)
        torch.cuda.synchronize()
        print(json.dumps({"omp_only": args.omp_only, "kernel": omp_kernel_name(h, 64, 256, 8),
                          "last_kernel_ms": h.last_kernel_ms()}))
        return

    if args.train_only:
        D = torch.from_numpy(synth.gaussian_dictionary(np.random.default_rng(1), 64, 256).astype(np.float32)).to(dev)
        labels = h.omp_code(D, Yt, 8)
        prop = h.proposer(Ws, bs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses = prop.train(Yt, labels, epochs=args.train_only, batch=1024, lr=1e-3, shuffle_seed=1)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        prop.close()
        print(json.dumps({"train_only": args.train_only, "ms": ms, "steps": args.train_only * (Ytr.shape[0] // 1024),
                          "losses": losses}))
        return

    def step():
        info = {}
        D, X, _, _ = h.split_merge_learn(Y, perm, w.offsets, w.K_local, w.s_local, w.K, w.iters_local,
                                         w.iters_merge, w.s_merge, w.s_final)
        info["phase_ms"] = h.phase_ms()
        info["final_kernel_ms"] = h.last_kernel_ms()
        # labels, and the plain residual of the training pairs that fixes the fallback threshold
        labels, rn_tr = h.omp_code(D, Yt, 8, res_norm=True)
        rms_tr = torch.sqrt((rn_tr.double() ** 2).mean())
        prop = h.proposer(Ws, bs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses = prop.train(Yt, labels, epochs=args.epochs, batch=1024, lr=1e-3, shuffle_seed=1)
        torch.cuda.synchronize()
        info["train_ms"] = (time.perf_counter() - t0) * 1e3
        t0 = time.perf_counter()
        Xp = h.omp_code(D, Ye, 8)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        info["plain_kernel_ms"] = h.last_kernel_ms()
        eps_fb = 1.1 * float(rms_tr.item())
        t0 = time.perf_counter()
        Xl, fb, nfb, _ = h.omp_code_proposed(prop, D, Ye, 8, 24, eps_fb)
        torch.cuda.synchronize()
        t_learn = time.perf_counter() - t0
        info.update(t_plain=t_plain, t_learn=t_learn, nfb=nfb, losses=losses, prop_ms=h.prop_phase_ms())
        info["D"], info["Xp"], info["Xl"], info["rms_tr"] = D, Xp, Xl, float(rms_tr.item())
        info["prop"] = prop
        return info

    for _ in range(args.warmup):
        step()["prop"].close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        infos.append(step())
        if len(infos) > 1:
            infos[-2]["prop"].close()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps

    last = infos[-1]
    D = last["D"]
    # representation error of both evaluation codings (FP64 on the GPU, plain torch)
    def rmse(X):
        Xd = X.dense(256).double()
        R = Ye.double() - Xd @ D.double()
        return float(torch.sqrt((R ** 2).mean()).item())
    r_plain, r_learn = rmse(last["Xp"]), rmse(last["Xl"])
    # learned vs plain along the fallback threshold (multiples of the training pairs' RMS plain
    # residual), after the timed steps: the equal-RMSE point is the largest multiplier whose
    # representation RMSE is within 1 % of the plain one
    prop = last["prop"]
    curve = []
    for mult in (1.1, 1.05, 1.02, 1.0, 0.95, 0.9, 0.85, 0.8):
        Xm, _, nfm, _ = h.omp_code_proposed(prop, D, Ye, 8, 24, mult * last["rms_tr"])
        torch.cuda.synchronize()
        ms = sum(h.prop_phase_ms())
        curve.append({"eps_mult": mult, "rmse_ratio": rmse(Xm) / r_plain, "fallback_rate": nfm / Yev.shape[0],
                      "learned_signals_per_s": Yev.shape[0] / (ms * 1e-3)})
    prop.close()
    n_local = int(w.N * (w.iters_local + 1))
    codings = n_local + w.N + Ytr.shape[0] + 2 * Yev.shape[0]
    value = codings / dt

    # roofline of the plain path's kernel: the fused OMP kernel, timed on the plain evaluation pass
    kms = float(np.mean([i["plain_kernel_ms"] for i in infos]))
    kname = omp_kernel_name(h, 64, 256, 8)
    f_sig = omp_flops_per_signal(64, 256, 8)
    achieved = f_sig * Yev.shape[0] / (kms * 1e-3) / 1e12
    plain_sps = Yev.shape[0] / (kms * 1e-3)
    prop_ms = last["prop_ms"]
    learned_sps = Yev.shape[0] / (sum(prop_ms) * 1e-3)
    out = {
        "metric": "signals sparse-coded/sec (m=64,K=256,s=8), learned vs plain, equal RMSE",
        "value": value,
        "unit": "signals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (OMP, MOD products f64, solve f64); bf16 proposer GEMMs",
        "data": "synthetic (Gaussian unit-atom dictionary, s=8 sparse codes, sigma=0.02 noise)",
        "config": {"workload": "split_merge_m64_K256_s8_N100000 + proposer_64-512-512-256_top24",
                   "N": w.N, "L": w.L, "n_local": 5000, "K": 256, "s": 8, "iters_local": w.iters_local,
                   "iters_merge": w.iters_merge, "s_merge": 4, "train_pairs": int(Ytr.shape[0]),
                   "eval_signals": int(Yev.shape[0]), "epochs": args.epochs, "codings_per_step": codings},
        "plain_signals_per_s": plain_sps,
        "learned_signals_per_s": learned_sps,
        "learned_vs_plain": learned_sps / plain_sps,
        "rmse_plain": r_plain,
        "rmse_learned": r_learn,
        "rmse_ratio": r_learn / r_plain,
        "fallback_rate": last["nfb"] / Yev.shape[0],
        "eps_fallback": "1.1 x RMS plain-OMP residual of the 200000 training pairs",
        "learned_vs_plain_curve": curve,
        "equal_rmse": None,
        "phase_ms": {"local": last["phase_ms"][0], "merge": last["phase_ms"][1],
                     "final": last["phase_ms"][2], "final_kernel": last["final_kernel_ms"],
                     "proposer_train": float(np.mean([i["train_ms"] for i in infos])),
                     "plain_eval_kernel": kms, "proposer_net_topk": prop_ms[0],
                     "proposer_restricted": prop_ms[1], "proposer_fallback": prop_ms[2]},
        "train_loss": last["losses"][-1] if last["losses"] else None,
        "roofline_proposer_training": train_roofline(widths, Ytr.shape[0] // 1024 * 1024 * args.epochs,
                                                     float(np.mean([i["train_ms"] for i in infos]))),
        "roofline": {"kernel": f"{kname} (plain OMP pass, N=100000)", "bound": "alu",
                     "achieved": achieved, "peak": FP32_PEAK, "unit": "TFLOP/s", "frac": achieved / FP32_PEAK,
                     "traffic": measured_traffic(kname), "traffic_unit": "bytes per launch (HBM read + write)",
                     "per_signal_flops": f_sig, "flops_note": ALGO_FLOPS_NOTE,
                     "alu_ops_per_signal": omp_alu_ops_per_signal(256, 8),
                     "per_signal_bytes": omp_bytes_per_signal(64, 8),
                     "kernel_ms": kms,
                     "mix_ceiling": {"peak": omp_mix_ceiling(64, 256, 8), "frac": achieved / omp_mix_ceiling(64, 256, 8),
                                     "unit": "TFLOP/s",
                                     "derivation": "correlations (2mK flops) as three FP16 products each at the "
                                                   "2.5 PFLOP/s FP16 matrix-core peak, the other flops at 78.6 "
                                                   "TFLOP/s (FP32 vector issue without packed FP32), combined "
                                                   "harmonically"}},
    }
    eq = [c for c in curve if c["rmse_ratio"] <= 1.01]
    if eq:
        best = max(eq, key=lambda c: c["eps_mult"])
        out["equal_rmse"] = {"eps_mult": best["eps_mult"], "rmse_ratio": best["rmse_ratio"],
                             "learned_vs_plain": best["learned_signals_per_s"] / plain_sps,
                             "fallback_rate": best["fallback_rate"]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_subsets, args.cpu_n, args.cpu_iters)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
