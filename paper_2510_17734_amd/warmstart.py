"""Learned warm start: a dense network that proposes starting cores.

The paper starts ALS from the initial guess of Sec. 5.2 (low-rank
completion, then Alg. "Randomized_LR_to_Butterfly"); random starts work
poorly there.  Here a network of four dense layers (width 512, ReLU) maps a
description of an instance -- its frequency, its geometry and a 64 x 64
binned summary of its observed entries -- to all butterfly cores at once.

Training data are completions the method itself produces: for each seeded
operator of the family (``workloads.warm_params``) ALS runs from a random
start on a shared sample of positions Omega_s, and the completed matrix's
values y_k at Omega_s are kept.  The training loss of instance k is
    1/2 ||X(cores(features_k)) - y_k||^2 / ||y_k||^2    on Omega_s,
which depends on the proposed cores only through the matrix they represent,
so the network is free to pick any gauge (the cores of a butterfly are
defined up to invertible r x r factors on every bond).  Its gradient with
respect to the cores is bfc_loss_gradient (the gradient contractions of
Sec. 5.1.2), back-propagated through the layers by the library's dense-layer
kernels and applied with ADAM, all in FP32; inference runs the same layers
with BF16 inputs and FP32 accumulation.  The last layer's bias starts at the
completed cores of the family's central operator, so the untrained network
already proposes a completion of a nearby operator.

The layers, the training step and the loss gradient run in libbfc.so; torch
holds device memory and forms the input features.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import api as bfc
from workloads import (WARM_HIST_BINS, WARM_L, WARM_N, WARM_R, gaussian_sketches,
                       green_geom_entries, observed_histogram, random_cores, sample_pairs,
                       warm_params)

N_FEATURES = 3 + WARM_HIST_BINS * WARM_HIST_BINS
CENTRAL = (2 * math.pi * 80.0, 1.125, 0.0)   # the family's central operator


def nnz_for(n: int) -> int:
    """Observed entries per instance: 8 n log2 n."""
    return 8 * n * int(round(math.log2(n)))


def features(omega: float, d: float, s: float, hist: torch.Tensor) -> torch.Tensor:
    """Network input: normalized (w, d, s) followed by the flattened histogram."""
    head = torch.tensor([(omega / (2 * math.pi) - 80.0) / 48.0, (d - 1.125) / 0.375, s / 0.25],
                        dtype=torch.float32, device=hist.device)
    return torch.cat([head, hist.reshape(-1).to(torch.float32)])


class WarmStartNet:
    """Dense layers dims[0] -> width -> ... -> dims[-1]; ReLU between layers."""

    def __init__(self, n_in: int, n_out: int, width: int = 512, depth: int = 4, seed: int = 0,
                 out_bias: torch.Tensor | None = None, out_scale: float = 0.01,
                 device="cuda:0"):
        g = torch.Generator(device="cpu").manual_seed(seed)
        dims = [n_in] + [width] * (depth - 1) + [n_out]
        self.W, self.b = [], []
        for l in range(depth):
            bound = math.sqrt(6.0 / dims[l]) * (out_scale if l == depth - 1 else 1.0)
            w = (torch.rand(dims[l], dims[l + 1], generator=g) * 2 - 1) * bound
            self.W.append(w.to(torch.float32).to(device).contiguous())
            self.b.append(torch.zeros(dims[l + 1], dtype=torch.float32, device=device))
        if out_bias is not None:
            self.b[-1].copy_(out_bias)
        self.params = self.W + self.b
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.t = 0
        self.depth = depth
        self._bf16 = None

    def forward_train(self, X: torch.Tensor):
        acts = [X]
        for l in range(self.depth):
            act = 1 if l < self.depth - 1 else 0
            acts.append(bfc.mlp_forward(acts[-1], self.W[l], self.b[l], act))
        return acts

    def backward(self, acts, d_out: torch.Tensor):
        gW, gb = [None] * self.depth, [None] * self.depth
        dY = d_out
        for l in reversed(range(self.depth)):
            act = 1 if l < self.depth - 1 else 0
            dX, gW[l], gb[l] = bfc.mlp_backward(acts[l], self.W[l], acts[l + 1], dY, act,
                                                need_dX=l > 0)
            dY = dX
        return gW + gb

    def step(self, grads, lr: float):
        self.t += 1
        for p, g_, m, v in zip(self.params, grads, self.m, self.v):
            bfc.mlp_adam(p, g_, m, v, self.t, lr)
        self._bf16 = None

    def infer_bf16(self, X: torch.Tensor) -> torch.Tensor:
        if self._bf16 is None:
            self._bf16 = [bfc.mlp_to_bf16(w) for w in self.W]
        xh = bfc.mlp_to_bf16(X)
        out = None
        for l in range(self.depth):
            last = l == self.depth - 1
            y, yh = bfc.mlp_forward_bf16(xh, self._bf16[l], self.b[l], 0 if last else 1,
                                         want_f32=last, want_bf16=not last)
            out, xh = y, yh
        return out


@dataclass
class Dataset:
    rows: torch.Tensor
    cols: torch.Tensor
    feats: torch.Tensor          # count x N_FEATURES
    targets: list                # completed matrix values at (rows, cols), complex128
    scales: list                 # 1 / ||y_k||^2
    completion_train_err: list


def _complete(prob, vals, n, L, r, seed, sweeps):
    rms = float(torch.sqrt(torch.mean(vals.abs() ** 2)))
    bfc.set_values(prob, vals)
    bfc.set_cores(prob, random_cores(n, L, r, seed, scale=rms * math.sqrt(r)))
    for _ in range(sweeps):
        bfc.sweep(prob)
    bfc.sync_status(prob)  # a training completion with failed solves is an error


def make_dataset(count: int, first_seed: int, *, sweeps: int = 40, pattern_seed: int = 77,
                 device="cuda:0", log=None, n=WARM_N, L=WARM_L, r=WARM_R) -> tuple:
    """Completions of `count` operators of the family (seeds first_seed...)
    on one shared sample Omega_s; returns (dataset, problem over Omega_s,
    central completion as interleaved float32 cores)."""
    rows, cols, _, _ = sample_pairs(n, nnz_for(n), 0, pattern_seed)
    rows_d = torch.as_tensor(rows, device=device)
    cols_d = torch.as_tensor(cols, device=device)
    cfg = bfc.Config(n=n, L=L, r=r, precision="c64")
    v0 = green_geom_entries(n, *CENTRAL, rows_d, cols_d)
    prob = bfc.init_cores(cfg, rows_d, cols_d, v0, random_cores(n, L, r, 1), device=device)
    _complete(prob, v0, n, L, r, 5, sweeps)
    central = torch.view_as_real(bfc.get_cores(prob)).reshape(-1).to(torch.float32).contiguous()
    feats, targets, scales, errs = [], [], [], []
    t0 = time.perf_counter()
    for k in range(count):
        w, d, s = warm_params(first_seed + k)
        vals = green_geom_entries(n, w, d, s, rows_d, cols_d)
        _complete(prob, vals, n, L, r, first_seed + k + 1000003, sweeps)
        y = bfc.predict_entries(prob, rows_d, cols_d)
        errs.append(float(torch.linalg.norm(y - vals) / torch.linalg.norm(vals)))
        targets.append(y)
        scales.append(1.0 / float(torch.sum(y.abs() ** 2)))
        feats.append(features(w, d, s, observed_histogram(n, rows_d, cols_d, vals)))
        if log and (k + 1) % 250 == 0:
            log(f"completions {k + 1}/{count} ({time.perf_counter() - t0:.1f} s), "
                f"median train err {np.median(errs):.2e}")
    ds = Dataset(rows_d, cols_d, torch.stack(feats).contiguous(), targets, scales, errs)
    return ds, prob, central


def train(net: WarmStartNet, ds: Dataset, prob, *, epochs: int, batch: int = 32,
          lr: float = 3e-4, seed: int = 0, log=None):
    """ADAM on the mean over the batch of each instance's relative loss."""
    rng = np.random.Generator(np.random.PCG64(seed))
    count = ds.feats.shape[0]
    history = []
    for ep in range(epochs):
        perm = rng.permutation(count)
        tot, nb = 0.0, 0
        for b0 in range(0, count, batch):
            idx = perm[b0:b0 + batch]
            X = ds.feats[torch.as_tensor(idx, device=ds.feats.device)].contiguous()
            acts = net.forward_train(X)
            out = acts[-1]
            d_out = torch.empty_like(out)
            # the batch's loss gradients, one call and one synchronization
            _, losses = bfc.loss_gradient_batch(
                prob, [ds.targets[k] for k in idx], [out[bi] for bi in range(len(idx))],
                [ds.scales[k] / len(idx) for k in idx], out=[d_out[bi] for bi in range(len(idx))])
            tot += sum(losses)
            net.step(net.backward(acts, d_out), lr)
            nb += 1
        history.append(tot / nb)
        if log:
            log(f"epoch {ep + 1}/{epochs}: mean relative loss {tot / nb:.4e} "
                f"(relative error ~{math.sqrt(2 * tot / nb):.3f})")
    return history


def _lowrank_guess(inst, prob_lr_cfg, device, sweeps=3, p=4):
    n, L, r = WARM_N, WARM_L, WARM_R
    rms = float(np.sqrt(np.mean(np.abs(inst["vals"]) ** 2)))
    lr = bfc.init_cores(prob_lr_cfg, inst["rows"], inst["cols"], inst["vals"],
                        random_cores(n, 0, r, inst["seed"] + 1, scale=rms * math.sqrt(r)),
                        device=device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(sweeps):
        bfc.sweep(lr)
    ab = bfc.get_cores(lr).reshape(2, n, r)
    flat = bfc.lowrank_to_butterfly(ab[0], ab[1], L, r, p, inst["sketches"], device=device)
    torch.cuda.synchronize()
    lr.close()
    return flat, time.perf_counter() - t0


def run_from_proposal(prob, proposal, guess, *, test, target: float = 1e-3,
                      max_sweeps: int = 150, judge_sweeps: int = 20, judge_err: float = 1e-3):
    """ALS from the network's proposal with the Sec. 5.2 guess as the fallback,
    judged by the ALS training residuals (never by the test entries).

    proposal: FP32 cores (bfc_set_cores_f32 layout); guess: a callable
    returning the guess's complex128 cores (computed only when needed).
    Sweeps run from the proposal until the test error reaches `target` (the
    evaluation's measure) or `judge_sweeps` sweeps are done.  If by then the
    training error (eq. (BF_convergence) on the observed entries) is not
    below `judge_err` -- or a solve failed, or it is not finite -- the guess
    is swept `judge_sweeps` times as well and the run continues from
    whichever start has the lower training error.  Every sweep counts
    against `max_sweeps`.  Returns sweeps to the target (None if missed),
    the final test error, whether the guess was tried and which start won."""
    bfc.set_cores_f32(prob, proposal)
    used, winner = 0, "learned"
    failed = False  # a solve failed during the current phase
    err, st = bfc.relative_error_status(prob, *test)

    def sweeps_until(limit):
        nonlocal used, err, failed
        while used < limit:
            bfc.sweep(prob)
            used += 1
            err, code = bfc.relative_error_status(prob, *test)
            failed = failed or code != 0
            if err <= target:
                return True
        return False

    def judged():  # the phase's training error; inf if a solve failed or it is not finite
        tr, code = bfc.relative_error_status(prob)
        return tr if (not failed and code == 0 and math.isfinite(tr)) else math.inf

    if sweeps_until(min(judge_sweeps, max_sweeps)):
        return {"sweeps": used, "final_err": err, "fallback_tried": False, "start": winner}
    tr_learned = judged()
    if tr_learned < judge_err:
        hit = sweeps_until(max_sweeps)
        return {"sweeps": used if hit else None, "final_err": err, "fallback_tried": False,
                "start": winner}
    kept = bfc.get_cores(prob).clone()
    bfc.set_cores(prob, guess())
    failed = False
    if sweeps_until(min(used + judge_sweeps, max_sweeps)):
        return {"sweeps": used, "final_err": err, "fallback_tried": True, "start": "lowrank"}
    tr_guess = judged()
    if tr_guess <= tr_learned:
        winner = "lowrank"
    else:
        bfc.set_cores(prob, kept)
        err, _ = bfc.relative_error_status(prob, *test)
    hit = err <= target or sweeps_until(max_sweeps)
    return {"sweeps": used if hit else None, "final_err": err, "fallback_tried": True,
            "start": winner}


def evaluate(net: WarmStartNet | None, seeds, *, target: float = 1e-3, max_sweeps: int = 150,
             device="cuda:0", log=None, starts=("learned", "lowrank", "random")):
    """Sweeps and time to `target` test error from each start, on instances
    with their own observed sets (8 n log2 n entries, 1000 test entries)."""
    n, L, r = WARM_N, WARM_L, WARM_R
    cfg = bfc.Config(n=n, L=L, r=r, precision="c64")
    lr_cfg = bfc.Config(n=n, L=0, r=r, precision="c64", reg_rel=1e-6)
    res = {s: [] for s in starts}
    fb = {"tried": 0, "lowrank_won": 0}
    for i, seed in enumerate(seeds):
        w, d, s_ = warm_params(seed)
        rows, cols, trows, tcols = sample_pairs(n, nnz_for(n), 1000, seed + 500009)
        vals = green_geom_entries(n, w, d, s_, rows, cols)
        tvals = green_geom_entries(n, w, d, s_, trows, tcols)
        inst = {"rows": rows, "cols": cols, "vals": vals, "seed": seed,
                "sketches": gaussian_sketches(n, L, r, 4, seed=seed + 3)}
        tr = (torch.as_tensor(trows, device=device), torch.as_tensor(tcols, device=device),
              torch.as_tensor(tvals, device=device))
        rms = float(np.sqrt(np.mean(np.abs(vals) ** 2)))
        rand = random_cores(n, L, r, seed + 7, scale=rms * math.sqrt(r))
        prob = bfc.init_cores(cfg, rows, cols, vals, rand, device=device)
        rows_d = torch.as_tensor(rows, device=device)
        cols_d = torch.as_tensor(cols, device=device)
        for start in starts:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if start == "learned+fallback":
                x = features(w, d, s_, observed_histogram(n, rows_d, cols_d,
                                                          torch.as_tensor(vals, device=device)))
                out = net.infer_bf16(x.reshape(1, -1).contiguous()).reshape(-1)
                run = run_from_proposal(prob, out, lambda: _lowrank_guess(inst, lr_cfg, device)[0],
                                        test=tr, target=target, max_sweeps=max_sweeps)
                torch.cuda.synchronize()
                spent = time.perf_counter() - t0
                fb["tried"] += run["fallback_tried"]
                fb["lowrank_won"] += run["start"] == "lowrank"
                res[start].append({"seed": seed, "start_err": float("nan"), "sweeps": run["sweeps"],
                                   "time_s": spent if run["sweeps"] else None,
                                   "final_err": run["final_err"], "start_s": 0.0,
                                   "fallback_tried": run["fallback_tried"],
                                   "winner": run["start"]})
                continue
            if start == "learned":
                x = features(w, d, s_, observed_histogram(n, rows_d, cols_d,
                                                          torch.as_tensor(vals, device=device)))
                out = net.infer_bf16(x.reshape(1, -1).contiguous())
                bfc.set_cores_f32(prob, out.reshape(-1))
                torch.cuda.synchronize()
                t_start = time.perf_counter() - t0
            elif start == "lowrank":
                flat, t_start = _lowrank_guess(inst, lr_cfg, device)
                bfc.set_cores(prob, flat)
            else:
                bfc.set_cores(prob, rand)
                t_start = 0.0
            e0 = bfc.relative_error(prob, *tr)
            torch.cuda.synchronize()
            spent, hit, err = t_start, None, e0
            for sw in range(max_sweeps):
                t1 = time.perf_counter()
                bfc.sweep(prob)
                torch.cuda.synchronize()
                spent += time.perf_counter() - t1
                err = bfc.relative_error(prob, *tr)
                if err <= target:
                    hit = sw + 1
                    break
            res[start].append({"seed": seed, "start_err": e0, "sweeps": hit,
                               "time_s": spent if hit else None, "final_err": err,
                               "start_s": t_start})
        prob.close()
        if log and (i + 1) % 25 == 0:
            log(f"evaluated {i + 1}/{len(seeds)}")
    if "learned+fallback" in res:
        res["fallback_counts"] = fb
    return res


def summarize(res, max_sweeps: int = 150):
    """Per start: instances reaching the target, median and mean sweeps (a
    miss counts as max_sweeps in the mean), mean time of those that reach
    it, median starting test error."""
    out = {}
    for start, rows in res.items():
        if start == "fallback_counts":
            out[start] = rows
            continue
        hits = [x for x in rows if x["sweeps"] is not None]
        out[start] = {
            "reached": len(hits), "instances": len(rows),
            "median_sweeps": float(np.median([x["sweeps"] if x["sweeps"] else max_sweeps
                                              for x in rows])) if rows else None,
            "mean_sweeps_capped": float(np.mean([x["sweeps"] or max_sweeps for x in rows]))
            if rows else None,
            "mean_time_to_target_s": float(np.mean([x["time_s"] for x in hits])) if hits else None,
            "median_start_test_err": float(np.nanmedian([x["start_err"] for x in rows]))
            if rows and not all(math.isnan(x["start_err"]) for x in rows) else None,
            "mean_start_s": float(np.mean([x["start_s"] for x in rows])) if rows else None,
        }
    return out


def evaluate_batched(net: WarmStartNet, seeds, *, chunk: int = 50, target: float = 1e-3,
                     max_sweeps: int = 150, device="cuda:0", log=None,
                     starts=("learned", "lowrank")):
    """The held-out instances swept together: per chunk of instances one
    batch (bfc_batch_sweep: one launch per kernel kind for all of them), the
    learned proposals inferred for the whole chunk at once.  Per start: the
    time until every instance of a chunk reaches `target` (or the cap),
    summed over chunks -- proposal, batch setup and sweeps, not the test-error
    checks -- the same time until 90% of a chunk has reached it (the cap when
    fewer do), and the instances reaching it."""
    n, L, r = WARM_N, WARM_L, WARM_R
    cfg = bfc.Config(n=n, L=L, r=r, precision="c64")
    lr_cfg = bfc.Config(n=n, L=0, r=r, precision="c64", reg_rel=1e-6)
    out = {s: {"time_s": 0.0, "reached": 0, "instances": 0, "sweeps": []} for s in starts}
    for c0 in range(0, len(seeds), chunk):
        insts, probs = [], []
        for seed in seeds[c0:c0 + chunk]:
            w, d, s_ = warm_params(seed)
            rows, cols, trows, tcols = sample_pairs(n, nnz_for(n), 1000, seed + 500009)
            vals = green_geom_entries(n, w, d, s_, rows, cols)
            tvals = green_geom_entries(n, w, d, s_, trows, tcols)
            rows_d = torch.as_tensor(rows, device=device)
            cols_d = torch.as_tensor(cols, device=device)
            vals_d = torch.as_tensor(vals, device=device)
            insts.append({"seed": seed, "rows": rows, "cols": cols, "vals": vals,
                          "w": w, "d": d, "s": s_,
                          "hist": observed_histogram(n, rows_d, cols_d, vals_d),
                          "sketches": gaussian_sketches(n, L, r, 4, seed=seed + 3),
                          "test": (torch.as_tensor(trows, device=device),
                                   torch.as_tensor(tcols, device=device),
                                   torch.as_tensor(tvals, device=device))})
            probs.append(bfc.init_cores(cfg, rows_d, cols_d, vals_d,
                                        random_cores(n, L, r, seed + 7), device=device))
        for start in starts:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if start == "learned+fallback":
                x = features(w, d, s_, observed_histogram(n, rows_d, cols_d,
                                                          torch.as_tensor(vals, device=device)))
                out = net.infer_bf16(x.reshape(1, -1).contiguous()).reshape(-1)
                run = run_from_proposal(prob, out, lambda: _lowrank_guess(inst, lr_cfg, device)[0],
                                        test=tr, target=target, max_sweeps=max_sweeps)
                torch.cuda.synchronize()
                spent = time.perf_counter() - t0
                fb["tried"] += run["fallback_tried"]
                fb["lowrank_won"] += run["start"] == "lowrank"
                res[start].append({"seed": seed, "start_err": float("nan"), "sweeps": run["sweeps"],
                                   "time_s": spent if run["sweeps"] else None,
                                   "final_err": run["final_err"], "start_s": 0.0,
                                   "fallback_tried": run["fallback_tried"],
                                   "winner": run["start"]})
                continue
            if start == "learned":
                X = torch.stack([features(x["w"], x["d"], x["s"], x["hist"]) for x in insts])
                prop = net.infer_bf16(X.contiguous())
                for i, p in enumerate(probs):
                    bfc.set_cores_f32(p, prop[i])
            else:
                for x, p in zip(insts, probs):
                    flat, _ = _lowrank_guess(x, lr_cfg, device)
                    bfc.set_cores(p, flat)
            b = bfc.batch_create(probs)
            torch.cuda.synchronize()
            spent = time.perf_counter() - t0
            done = [None] * len(probs)
            t90 = None
            for sw in range(max_sweeps):
                t1 = time.perf_counter()
                bfc.batch_sweep(b)
                torch.cuda.synchronize()
                spent += time.perf_counter() - t1
                for i, (x, p) in enumerate(zip(insts, probs)):
                    if done[i] is None and bfc.relative_error(p, *x["test"]) <= target:
                        done[i] = sw + 1
                hits = sum(v is not None for v in done)
                if t90 is None and hits >= 0.9 * len(done):
                    t90 = spent
                if hits == len(done):
                    break
            b.close()
            o = out[start]
            o["time_s"] += spent
            o["time_to_90pct_s"] = (o.get("time_to_90pct_s") or 0.0) + (t90 if t90 else spent)
            o["reached"] += sum(v is not None for v in done)
            o["instances"] += len(done)
            o["sweeps"].append(max(v or max_sweeps for v in done))
        for p in probs:
            p.close()
        if log:
            log(f"batched evaluation {min(c0 + chunk, len(seeds))}/{len(seeds)}")
    for o in out.values():
        o["time_s"] = round(o["time_s"], 4)
        o["time_to_90pct_s"] = round(o.get("time_to_90pct_s", 0.0), 4)
        o["sweeps_until_chunk_done"] = o.pop("sweeps")
    return out


def precision_check(net: WarmStartNet, seeds, *, sweeps: int = 60, device="cuda:0"):
    """Complex64 sweeps (FP32 contractions and Grams, FP64 solves) against the
    same method in FP64 (complex128 with the complex64 modes' regularization
    floor 2^-20, so lambda is identical) from the same learned proposal, per
    held-out instance: the test errors after `sweeps` sweeps and their gap
    |e_c64 - e_fp64| in relative-error units.  Complex128 at its own floor
    (lambda = 1e-10 tau, a less regularized method) is reported beside them."""
    n, L, r = WARM_N, WARM_L, WARM_R
    rows_out = []
    runs = (("c64", "c64", 0.0), ("fp64", "c128", 2.0 ** -20), ("fp64_own_floor", "c128", 0.0))
    for seed in seeds:
        w, d, s_ = warm_params(seed)
        rows, cols, trows, tcols = sample_pairs(n, nnz_for(n), 1000, seed + 500009)
        vals = green_geom_entries(n, w, d, s_, rows, cols)
        tvals = green_geom_entries(n, w, d, s_, trows, tcols)
        rows_d = torch.as_tensor(rows, device=device)
        cols_d = torch.as_tensor(cols, device=device)
        vals_d = torch.as_tensor(vals, device=device)
        test = (torch.as_tensor(trows, device=device), torch.as_tensor(tcols, device=device),
                torch.as_tensor(tvals, device=device))
        x = features(w, d, s_, observed_histogram(n, rows_d, cols_d, vals_d))
        prop = net.infer_bf16(x.reshape(1, -1).contiguous()).reshape(-1)
        errs = {}
        for name, prec, floor in runs:
            p = bfc.init_cores(bfc.Config(n=n, L=L, r=r, precision=prec, reg_floor=floor),
                               rows_d, cols_d, vals_d, random_cores(n, L, r, seed + 7),
                               device=device)
            bfc.set_cores_f32(p, prop)
            for _ in range(sweeps):
                bfc.sweep(p)
            errs[name] = bfc.relative_error(p, *test)
            p.close()
        rows_out.append(dict(seed=seed, gap=abs(errs["c64"] - errs["fp64"]), **errs))
    gaps = [x["gap"] for x in rows_out]
    return {"instances": len(rows_out), "sweeps": sweeps,
            "max_gap_to_fp64": max(gaps), "median_gap_to_fp64": float(np.median(gaps)),
            "within_1e-4": sum(g <= 1e-4 for g in gaps),
            "median_c64_test_err": float(np.median([x["c64"] for x in rows_out])),
            "median_fp64_test_err": float(np.median([x["fp64"] for x in rows_out])),
            "median_fp64_own_floor_test_err":
                float(np.median([x["fp64_own_floor"] for x in rows_out]))}
