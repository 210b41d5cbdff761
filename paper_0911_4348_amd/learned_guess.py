"""Learned initial guess for the second-Born SCF: data, training, evaluation.

A float32 MLP (26 -> 256 -> 256 -> 256 -> 1, tanh hidden layers; the library's
negf_mlp_* kernels) maps per-sample features of (i, j, tau) and of the
potential's nuclei to dG_ij(tau) = G_ij(tau) - G0_ij(tau), where G is the
converged second-Born Green's function and G0 the HF one. The SCF then starts
from G0 + sym(dG) instead of G0 (negf_opts_t.guess_params); the HF start stays
the fallback, and both starts run to the same stopping rule so their iteration
counts and wall times compare at equal final energy.

Workflow (all compute in the library's HIP kernels; torch only holds device
memory and shuffles sample indices):
  generate()  converged G for seeded random potentials (batched SCF), sampled
              targets dG at seeded (i, j, tau) points;
  train()     Adam on mini-batches with negf_mlp_train_step;
  evaluate()  SCF from the HF start and from the learned start on held-out
              potentials: iterations, wall time, final energies.
Run as ``python -m paper_0911_4348_amd.learned_guess {generate,train,evaluate}``.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
WEIGHTS = os.path.join(HERE, "data", "mlp_guess_nb199.npz")

# network shape: input features, hidden width; must agree with the library
D_IN, HIDDEN = 26, 256
LAYERS = [(D_IN, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, 1)]
N_SAMPLES = 4096          # sampled (i <= j, tau) points per training system
TRAIN_SEEDS = range(0, 2000)
HELD_OUT_SEEDS = range(100000, 100256)


def _imports():
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import torch
    import paper_0911_4348_amd as negf
    import workloads as W
    return torch, negf, W


def sample_points(seed: int, x: np.ndarray, n_tau: int, count: int = N_SAMPLES):
    """Seeded sample points (i <= j, q): each index half uniform over the grid,
    half uniform over the nodes with |x| < 10 (where the nuclei sit); tau
    half uniform, half within 64 points of either end."""
    rng = np.random.default_rng(10_000_019 + seed)
    n = len(x)
    core = np.nonzero(np.abs(x) < 10.0)[0]

    def idx():
        a = rng.integers(0, n, size=count)
        b = core[rng.integers(0, len(core), size=count)]
        return np.where(rng.random(count) < 0.5, a, b)

    i, j = idx(), idx()
    ii, jj = np.minimum(i, j), np.maximum(i, j)
    qu = rng.integers(0, n_tau, size=count)
    qe = rng.integers(0, 64, size=count)
    qe = np.where(rng.random(count) < 0.5, qe, n_tau - 1 - qe)
    qq = np.where(rng.random(count) < 0.5, qu, qe)
    return ii.astype(np.int32), jj.astype(np.int32), qq.astype(np.int32)


def _dev_setup(torch, negf, sysd):
    x, Wt, T, v, V = negf.fedvr_build_system(sysd)
    tau = negf.tau_grid_system(sysd)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return x, d(x), d(v), d(tau), (T, v, V)


def generate(seeds, tol=1e-5, refine_tol=1e-9, dtype="bf16", chunk=16, max_iter=150, log=print, save_path=None):
    """Converged G for each seeded random potential on the n_b = 199 grid, and the
    targets dG at its sample points. Returns float32 [len(seeds), N_SAMPLES].
    The batched SCF runs the low-precision loop to tol and then float64 steps
    until the contraction-aware bound on |E - E_inf| is below refine_tol, so the
    targets are those of the float64 fixed point. Systems not converged within
    max_iter steps (the batch waits for its slowest member) are excluded."""
    torch, negf, W = _imports()
    ctx = negf.Context(0)
    seeds = list(seeds)
    out = np.zeros((len(seeds), N_SAMPLES), dtype=np.float32)
    t0 = time.perf_counter()
    iters = []
    for c0 in range(0, len(seeds), chunk):
        sub = seeds[c0:c0 + chunk]
        systems = [W.random_potential_system(s) for s in sub]
        res = negf.scf_batched(ctx, systems, tol=tol, dtype=dtype, refine_tol=refine_tol, conv=negf.CONV_FFT,
                               max_iter=max_iter, allow_noconv=True, tune=True, stop="contraction")
        # G0 of each system: batched HF (same grid) and the HF Green's function
        mats = [negf.fedvr_build_system(s) for s in systems]
        d = lambda a: torch.from_numpy(np.ascontiguousarray(np.stack(a))).cuda()
        eps, Cm, rho, S0, mu, E, it = negf.hf_batched(ctx, d([m[2] for m in mats]), d([m[3] for m in mats]),
                                                      d([m[4] for m in mats]), systems[0].n_elec,
                                                      systems[0].sigma, systems[0].beta, allow_noconv=True)
        tau = negf.tau_grid_system(systems[0])
        for k, (s, r) in enumerate(zip(systems, res)):
            hfs = negf.HFState(eps[k], Cm[k], rho[k], S0[k], float(mu[k]), float(E[k]), int(it[k]))
            G0 = negf.g0_build(ctx, hfs, tau, s.beta)
            ii, jj, qq = sample_points(sub[k], mats[k][0], s.n_tau)
            di = lambda a: torch.from_numpy(a).cuda()
            x_d = torch.from_numpy(np.ascontiguousarray(mats[k][0])).cuda()
            tau_d = torch.from_numpy(tau).cuda()
            if r.status != negf.OK:
                # excluded from training (NaN row): the plain SCF did not converge for it
                out[c0 + k] = np.nan
                log(f"generate: system {sub[k]} stopped with status {r.status} after {r.iters} steps")
            else:
                t = negf.mlp_targets(ctx, s, x_d, tau_d, r.G, G0, 1.0, di(ii), di(jj), di(qq))
                out[c0 + k] = t.cpu().numpy()
                iters.append(r.iters)
            del G0
        del res
        log(f"generate: {c0 + len(sub)}/{len(seeds)} systems, {time.perf_counter() - t0:.1f} s, "
            f"mean SCF steps {np.mean(iters):.1f}")
        if save_path:
            np.save(save_path, out[:c0 + len(sub)])
    ctx.close()
    return out


def convert_raw(seeds, raw, log=print):
    """Targets stored as plain dG (out_scale 1, no envelope) -> dG / e at the same
    sample points (e from negf_mlp_envelope); NaN rows stay NaN."""
    torch, negf, W = _imports()
    ctx = negf.Context(0)
    out = np.array(raw, dtype=np.float32, copy=True)
    base = W.config_sigma_bench()
    for k, seed in enumerate(seeds):
        if not np.all(np.isfinite(out[k])):
            continue
        s = W.random_potential_system(seed, base)
        x, x_d, v_d, tau_d, _ = _dev_setup(torch, negf, s)
        ii, jj, qq = sample_points(seed, x, s.n_tau)
        di = lambda a: torch.from_numpy(a).cuda()
        e = negf.mlp_envelope(ctx, s, x_d, tau_d, di(ii), di(jj), di(qq)).cpu().numpy()
        out[k] = out[k] / e
    ctx.close()
    log(f"convert: {len(seeds)} systems")
    return out


def features_for(ctx, torch, negf, W, seeds):
    """Feature rows [len(seeds) * N_SAMPLES, 26] on the device."""
    base = W.config_sigma_bench()
    F = torch.empty((len(seeds) * N_SAMPLES, D_IN), dtype=torch.float32, device="cuda")
    for k, seed in enumerate(seeds):
        s = W.random_potential_system(seed, base)
        x, x_d, v_d, tau_d, _ = _dev_setup(torch, negf, s)
        ii, jj, qq = sample_points(seed, x, s.n_tau)
        di = lambda a: torch.from_numpy(a).cuda()
        F[k * N_SAMPLES:(k + 1) * N_SAMPLES] = negf.mlp_features(ctx, s, x_d, v_d, tau_d, di(ii), di(jj), di(qq))
    return F


def train(seeds, targets, epochs=40, batch=8192, lr=1e-3, lr_min=2e-5, seed=0, val_frac=0.05, log=print):
    """Adam with cosine learning-rate decay; the last val_frac of the systems is
    kept out of the updates and reported as validation loss. Returns
    (params float32 numpy, out_scale, history)."""
    torch, negf, W = _imports()
    ctx = negf.Context(0)
    seeds = list(seeds)
    y = np.asarray(targets, dtype=np.float32).reshape(-1)
    out_scale = float(np.std(y)) or 1.0
    F = features_for(ctx, torch, negf, W, seeds)
    T = torch.from_numpy(y / out_scale).cuda()
    n_val = max(1, int(len(seeds) * val_frac)) * N_SAMPLES
    n_tr = F.shape[0] - n_val
    params = torch.from_numpy(W.mlp_init(LAYERS, seed).astype(np.float32)).cuda()
    assert params.numel() == negf.mlp_param_count()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    steps_per_epoch = n_tr // batch
    total = epochs * steps_per_epoch
    step = 0
    hist = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(n_tr, generator=gen, device="cuda")
        for b in range(steps_per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            step += 1
            lr_t = lr_min + 0.5 * (lr - lr_min) * (1.0 + np.cos(np.pi * step / total))
            negf.mlp_train_step(ctx, params, m, v, step, lr_t, F.index_select(0, idx).contiguous(),
                                T.index_select(0, idx).contiguous(), want_loss=False)
        def mse(lo, hi):
            acc = 0.0
            for c in range(lo, hi, 1 << 20):
                e = min(hi, c + (1 << 20))
                yv = negf.mlp_forward(ctx, params, F[c:e])
                acc += float(torch.sum((yv - T[c:e]) ** 2).item())
            return acc / (hi - lo)
        tr, val = mse(0, n_tr), mse(n_tr, F.shape[0])
        var_tr = float(torch.mean(T[:n_tr] ** 2).item())
        var = float(torch.mean(T[n_tr:] ** 2).item())
        hist.append({"epoch": ep + 1, "train_loss": tr, "train_rel": tr / var_tr, "val_loss": val,
                     "val_rel": val / var, "s": round(time.perf_counter() - t0, 2)})
        log(f"train: epoch {ep + 1}/{epochs} train {tr:.4e} (rel {tr / var_tr:.3f}) val {val:.4e} "
            f"(rel {val / var:.3f}) {time.perf_counter() - t0:.1f} s")
    p = params.cpu().numpy()
    ctx.close()
    return p, out_scale, hist


def save(path, params, out_scale, info):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, params=params.astype(np.float32), out_scale=np.float64(out_scale),
             info=np.frombuffer(json.dumps(info).encode(), dtype=np.uint8))


def load(path=WEIGHTS):
    z = np.load(path, allow_pickle=False)
    info = json.loads(bytes(z["info"]).decode())
    return z["params"].astype(np.float32), float(z["out_scale"]), info


def _time_to(log_rows, wall_s, tol, E_ref):
    """Steps and wall time until |E_k - E_ref| < tol first holds, from an SCF log
    whose records carry per-iteration milliseconds; set-up time (HF, starting G)
    is the wall time not covered by the records."""
    ms = [r["ms"] for r in log_rows]
    setup = wall_s - sum(ms) * 1e-3
    for k, r in enumerate(log_rows):
        if abs(r["E"] - E_ref) < tol:
            return k, setup + sum(ms[:k + 1]) * 1e-3
    return len(ms) - 1, wall_s


def evaluate(seeds, path=WEIGHTS, tol=1e-6, ref_tol=1e-10, dtype="f64", log=print):
    """Per held-out potential, three float64 runs with the library's
    contraction-aware stopping rule: the HF start to ref_tol gives E_ref; the HF
    start and the learned start to tol give the compared steps and wall times
    (HF, guess and set-up included), each with its final |E - E_ref|, and the
    steps and time until |E_k - E_ref| < tol first held."""
    torch, negf, W = _imports()
    ctx = negf.Context(0)
    params, scale, _ = load(path)
    P = torch.from_numpy(params).cuda()
    kw = dict(dtype=dtype, conv=negf.CONV_FFT, want_G=False, max_iter=600, allow_noconv=True, stop="contraction")
    rows = []
    # one untimed run for kernel loading and table set-up
    negf.scf(ctx, W.random_potential_system(int(list(seeds)[0])), tol=tol, **kw)
    for seed in seeds:
        s = W.random_potential_system(int(seed))
        ref = negf.scf(ctx, s, tol=ref_tol, **kw)
        if ref.status != negf.OK:
            log(f"evaluate {seed}: HF-started SCF failed (status {ref.status}); system skipped")
            rows.append({"seed": int(seed), "skipped": True, "status": ref.status})
            continue
        E_ref = ref.E
        runs = {}
        for name, extra in (("hf_start", {}), ("learned", {"guess": P, "guess_scale": scale})):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = negf.scf(ctx, s, tol=tol, **kw, **extra)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            k_acc, s_acc = _time_to(r.log, wall, tol, E_ref)
            runs[name] = {"iters": r.iters, "s": wall, "err": abs(r.E - E_ref), "status": r.status,
                          "iters_to_acc": k_acc, "s_to_acc": s_acc}
        a, b = runs["hf_start"], runs["learned"]
        rows.append({"seed": int(seed), "E_ref": E_ref, "E_hf": ref.hf_E, "status_learned": b["status"],
                     "iters_hf_start": a["iters"], "s_hf_start": a["s"], "err_hf_start": a["err"],
                     "iters_learned": b["iters"], "s_learned": b["s"], "err_learned": b["err"],
                     "iters_to_acc_hf_start": a["iters_to_acc"], "s_to_acc_hf_start": a["s_to_acc"],
                     "iters_to_acc_learned": b["iters_to_acc"], "s_to_acc_learned": b["s_to_acc"]})
        log(f"evaluate {seed}: HF start {a['iters']} steps {a['s']:.2f} s err {a['err']:.1e}; learned "
            f"{b['iters']} steps {b['s']:.2f} s err {b['err']:.1e}")
    ctx.close()
    return rows


def summarize(rows):
    skipped = [r["seed"] for r in rows if r.get("skipped")]
    rows = [r for r in rows if not r.get("skipped")]
    g = lambda k: np.array([r[k] for r in rows], float)
    ia, ib = g("iters_hf_start"), g("iters_learned")
    ta, tb = g("s_hf_start"), g("s_learned")
    aa, ab = g("iters_to_acc_hf_start"), g("iters_to_acc_learned")
    sa, sb = g("s_to_acc_hf_start"), g("s_to_acc_learned")
    return {"systems": len(rows), "skipped_seeds": skipped,
            "stopping_rule": {"mean_iters_hf_start": ia.mean(), "mean_iters_learned": ib.mean(),
                              "median_iters_hf_start": float(np.median(ia)),
                              "median_iters_learned": float(np.median(ib)),
                              "total_s_hf_start": ta.sum(), "total_s_learned": tb.sum(),
                              "speedup": ta.sum() / tb.sum(), "systems_with_fewer_iters": int((ib < ia).sum()),
                              "systems_with_more_iters": int((ib > ia).sum()),
                              "max_err_hf_start": g("err_hf_start").max(),
                              "max_err_learned": g("err_learned").max(),
                              "median_err_hf_start": float(np.median(g("err_hf_start"))),
                              "median_err_learned": float(np.median(g("err_learned"))),
                              "systems_hf_err_above_tol": int((g("err_hf_start") > 1e-6).sum()),
                              "systems_learned_err_above_tol": int((g("err_learned") > 1e-6).sum())},
            "to_accuracy": {"mean_iters_hf_start": aa.mean(), "mean_iters_learned": ab.mean(),
                            "total_s_hf_start": sa.sum(), "total_s_learned": sb.sum(),
                            "speedup": sa.sum() / sb.sum()}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["generate", "convert", "train", "evaluate"])
    ap.add_argument("--first", type=int, default=0)
    ap.add_argument("--count", type=int, default=len(TRAIN_SEEDS))
    ap.add_argument("--data", default=None, help="targets file (.npy): written by generate, read by train")
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--report", default=None)
    args = ap.parse_args()
    log = lambda m: print(m, flush=True)
    if args.cmd == "generate":
        seeds = list(TRAIN_SEEDS)[args.first:args.first + args.count]
        t = generate(seeds, log=log, save_path=args.data)
        np.save(args.data, t)
    elif args.cmd == "convert":
        raw = np.load(args.data, allow_pickle=False)
        seeds = list(TRAIN_SEEDS)[args.first:args.first + raw.shape[0]]
        np.save(args.out, convert_raw(seeds, raw, log=log))
    elif args.cmd == "train":
        parts = [np.load(p, allow_pickle=False) for p in args.data.split(",")]
        t = np.concatenate(parts)
        seeds = np.array(list(TRAIN_SEEDS)[:t.shape[0]])
        ok = np.all(np.isfinite(t), axis=1)
        log(f"train: {int(ok.sum())} systems, {int((~ok).sum())} excluded: {seeds[~ok].tolist()}")
        p, scale, hist = train(seeds[ok].tolist(), t[ok], epochs=args.epochs, log=log)
        save(args.out, p, scale, {"train_seeds": [int(seeds[0]), int(seeds[-1])],
                                  "excluded_seeds": seeds[~ok].tolist(), "samples_per_system": N_SAMPLES,
                                  "history": hist})
    else:
        seeds = list(HELD_OUT_SEEDS)[args.first:args.first + args.count]
        rows = evaluate(seeds, path=args.out, log=log)
        summ = summarize(rows)
        log(json.dumps(summ, default=float))
        if args.report:
            with open(args.report, "w") as f:
                json.dump({"summary": summ, "rows": rows}, f, default=float)


if __name__ == "__main__":
    main()
