"""Learned initial guess for GMRES on the 64 x 64 P1 SIPG family of
diffusion-convection-reaction problems (parameters drawn as for the batched
workload).

Pipeline (every step runs in the library's kernels; this module moves
arguments and buffers):
  features (the 23 instance parameters) -> multilayer perceptron (BF16
  products, FP32 accumulation) -> u_h means on a coarse 32 x 32 grid of cells
  -> prolongation to DG P1 coefficients on the 64 x 64 mesh -> GMRES with that
  initial guess; the true FP64 residual rejects a guess worse than zero.

The network is trained on solutions the method itself computes (batched
assemble + solve to relative residual 1e-10).  Training targets are the cell
means of u_h: with the orthonormal basis the mean of u_h over a triangle is
sqrt(2) times its first coefficient, and the 8 triangles of a coarse cell have
equal area.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import api as A
from . import workloads as W

FINE = 64
COARSE = 32
N_DOFS = 2 * FINE * FINE * 3


def instances(count, seed):
    return W.sample_instances(count, seed=seed, fixed_N=FINE, fixed_k=1)


def features(insts):
    return np.stack([i.features() for i in insts]).astype(np.float32)


def coarse_means(x, n=FINE, nc=COARSE):
    """x: [B, 6 n^2] P1 coefficients of the structured n x n mesh (element
    2 (j n + i) + t) -> [B, nc^2] means of u_h over the coarse cells, cell
    index cj * nc + ci."""
    x = np.asarray(x)
    B = x.shape[0]
    c0 = x.reshape(B, n, n, 2, 3)[..., 0] * math.sqrt(2.0)
    r = n // nc
    return c0.reshape(B, nc, r, nc, r, 2).mean(axis=(2, 4, 5)).reshape(B, nc * nc)


class Family:
    """The fixed 64 x 64 mesh and batched solves of a list of instances."""

    def __init__(self, insts, mixed, lockstep_min_dofs=0, log=None, **opts):
        self.insts = insts
        self.mesh_arrays = W.structured_mesh(FINE)
        self.batch = A.Batch([(self.mesh_arrays, A.instance_problem(i)) for i in insts], mixed=mixed,
                             rel_tol=1e-10, inner_tol=opts.pop("inner_tol", 1e-5),
                             lockstep_min_dofs=lockstep_min_dofs, log=log, **opts)
        assert self.batch.n_dofs == len(insts) * N_DOFS
        self.log = log

    def solve(self, x=None, rep=None, stream=None):
        """x: [B, N_DOFS] FP64 initial guesses (zero if None), solutions on return."""
        if x is None:
            x = torch.zeros(len(self.insts), N_DOFS, dtype=torch.float64, device="cuda")
        if rep is None:
            _, rep = self.batch.alloc()
        self.batch.run(x.view(-1), rep, stream)
        self.batch.wait(self.log, stream=stream)
        return x, rep


def fold_standardisation(params, widths, mu, sd, yscale):
    """Parameters of the same network acting on raw features and producing raw
    targets: W1 <- W1 / sd, b1 <- b1 - W1 (mu / sd); W_L <- yscale W_L,
    b_L <- yscale b_L."""
    p = np.array(params, dtype=np.float64)
    o = 0
    L = len(widths) - 1
    for l in range(L):
        k, n = widths[l], widths[l + 1]
        Wl = p[o:o + n * k].reshape(n, k)
        bl = p[o + n * k:o + n * k + n]
        if l == 0:
            bl -= Wl @ (mu / sd)
            Wl /= sd[None, :]
        if l == L - 1:
            Wl *= yscale
            bl *= yscale
        o += n * k + n
    return p.astype(np.float32)


def generate(count, seed, chunk=2048, log=None):
    """Training data from the method itself: features [count, 23] and the
    coarse cell means of the solutions [count, COARSE^2] (batched assemble +
    mixed-precision solve to relative residual 1e-10 from the zero guess)."""
    insts = instances(count, seed)
    X = features(insts)
    Y = np.empty((count, COARSE * COARSE), np.float32)
    iters = np.empty(count, np.int32)
    t0 = time.perf_counter()
    for s in range(0, count, chunk):
        part = insts[s:s + chunk]
        fam = Family(part, mixed=True)
        x, rep = fam.solve()
        R = A.Batch.reports(rep)
        bad = np.flatnonzero(R["status"] != 0)
        if len(bad):
            raise RuntimeError("training solve %d did not converge: %s" % (s + bad[0], R[bad[0]]))
        Y[s:s + len(part)] = coarse_means(x.cpu().numpy())
        iters[s:s + len(part)] = R["iters"]
        if log:
            log("dataset: %d/%d solves (%.1f s)" % (s + len(part), count, time.perf_counter() - t0))
        del fam, x, rep
        torch.cuda.empty_cache()
    return X, Y, iters


N_HEAD = 7  # log10 eps, cos, sin, |b|, b_x, b_y, alpha; then 4 x (c_x, c_y, width, amplitude)


def _augment_index(B, g):
    """Per sample, a random order of the 4 Gaussians (the solution does not
    depend on it): column gather indices [B, 23]."""
    order = torch.argsort(torch.rand(B, 4, device="cuda", generator=g), dim=1)
    cols = N_HEAD + (order[:, :, None] * 4 + torch.arange(4, device="cuda")[None, None, :]).reshape(B, 16)
    head = torch.arange(N_HEAD, device="cuda")[None, :].expand(B, N_HEAD)
    return torch.cat([head, cols], dim=1)


def train(X, Y, epochs=60, batch=256, lr=1e-3, lr_end=1e-5, seed=0, n_val=1000, augment=True, log=None):
    """Trains the perceptron on (X, Y) with the library's forward / backward /
    Adam kernels: inputs standardised per feature, targets scaled by their
    standard deviation, mean squared error, cosine learning-rate decay.  With
    `augment`, each minibatch sample gets a random order of its Gaussians and
    a random common sign of their amplitudes and of the target (the problem is
    linear in f).  Returns the model dict (raw parameters and the
    standardisation)."""
    widths = W.mlp_widths()
    mu = X[n_val:].mean(axis=0).astype(np.float64)
    sd = X[n_val:].std(axis=0).astype(np.float64)
    if augment:  # statistics shared by the 4 Gaussian slots, amplitude mean 0
        g4 = X[n_val:, N_HEAD:].reshape(-1, 4, 4)
        mu[N_HEAD:] = np.tile(g4.mean(axis=(0, 1)), 4)
        sd[N_HEAD:] = np.tile(g4.std(axis=(0, 1)), 4)
        mu[N_HEAD + 3::4] = 0.0
    sd[sd == 0] = 1.0
    ys = float(Y[n_val:].std())
    Xn = ((X - mu) / sd).astype(np.float32)
    Yn = (Y / ys).astype(np.float32)
    Xv, Yv = torch.from_numpy(Xn[:n_val]).cuda(), torch.from_numpy(Yn[:n_val]).cuda()
    Xt, Yt = torch.from_numpy(Xn[n_val:]).cuda(), torch.from_numpy(Yn[n_val:]).cuda()
    ntr = Xt.shape[0]
    net = A.MLP(widths, max(batch, n_val), W.mlp_init(widths, seed))
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    steps = ntr // batch
    total = epochs * steps
    hist = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(ntr, device="cuda", generator=g)
        for s in range(steps):
            idx = perm[s * batch:(s + 1) * batch]
            xb, yb = Xt[idx], Yt[idx]
            if augment:
                xb = torch.gather(xb, 1, _augment_index(batch, g))
                sgn = torch.where(torch.rand(batch, 1, device="cuda", generator=g) < 0.5, -1.0, 1.0)
                xb[:, N_HEAD + 3::4] *= sgn
                yb = yb * sgn
            net.forward(xb)
            _, dy = net.loss_mse(yb)
            net.backward(dy)
            t = ep * steps + s
            net.adam_step(lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * t / total)))
        lt = float(net.loss_mse(yb)[0].item())
        net.forward(Xv)
        lv = float(net.loss_mse(Yv)[0].item())
        hist.append((ep, lt, lv))
        if log and (ep % 5 == 4 or ep == epochs - 1):
            log("epoch %d: train mse %.4g  validation mse %.4g (%.1f s)" % (ep + 1, lt, lv, time.perf_counter() - t0))
    p, _ = net.params()
    return {"params": p.cpu().numpy(), "mu": mu, "sd": sd, "yscale": np.float64(ys),
            "widths": np.asarray(widths, np.int32), "history": np.asarray(hist, np.float64)}


def save(model, path):
    np.savez(path, **model)


def load(path):
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


class WarmStart:
    """Inference: raw features -> coarse cell means -> DG P1 initial guess, on
    the device (the standardisation is folded into the first and last layers)."""

    def __init__(self, model, max_batch, mode=1):
        widths = [int(w) for w in model["widths"]]
        folded = fold_standardisation(model["params"], widths, model["mu"], model["sd"], float(model["yscale"]))
        self.net = A.MLP(widths, max_batch, folded)
        self.mesh = A.Mesh.from_arrays(W.structured_mesh(FINE), 1)
        self.mode = mode

    def coarse(self, feats: torch.Tensor, stream=None):
        return self.net.forward(feats, stream=stream)

    def guess(self, feats: torch.Tensor, x: torch.Tensor = None, stream=None):
        """feats [B, 23] FP32 on the device -> x [B, N_DOFS] FP64."""
        B = feats.shape[0]
        if x is None:
            x = torch.empty(B, N_DOFS, dtype=torch.float64, device="cuda")
        c = self.coarse(feats, stream)
        A.warmstart_prolong(self.mesh, c, COARSE, self.mode, x, stream)
        return x


# How the true residual judges a learned guess.  A coarse guess is rough on
# the fine mesh (jumps, gradient kinks, layers it cannot resolve), so its
# residual norm exceeds ||F|| on this family even when its error is small: the
# exact coarse means of method solutions, prolonged bilinearly, have residuals
# of 1.9 to 4.5 ||F||.  The default judge (reject a guess worse than zero)
# therefore falls back to the zero guess for nearly every instance, and the
# learned path never costs iterations.  NO_JUDGE keeps every finite guess; it is
# evaluated only to show what the guess would do to GMRES without the judge.
NO_JUDGE = math.inf

# (name, mixed cycles, initial guess, judge limit): the guess is zero, the
# network's ("net"), or the exact cell means of the solution itself ("exact":
# what a perfect coarse predictor would give; needs the "fp64" form first)
FORMS = (("fp64", False, None, 0.0), ("mixed", True, None, 0.0), ("fp64+learned", False, "net", 0.0),
         ("mixed+learned", True, "net", 0.0), ("mixed+learned(no judge)", True, "net", NO_JUDGE),
         ("mixed+exact coarse(no judge)", True, "exact", NO_JUDGE))
# the forms of the comparison "learned + mixed vs plain FP64"
HEADLINE_FORMS = FORMS[:2] + FORMS[3:4]


def evaluate(model, count=512, seed=2, reps=3, forms=FORMS, log=None, lockstep_block=0):
    """Held-out instances: GMRES iterations and wall time to relative residual
    1e-10 for the zero and the learned guess, FP64 and mixed cycles.  The
    learned forms' time includes the network and the prolongation."""
    insts = instances(count, seed)
    feats = torch.from_numpy(features(insts)).cuda()
    ws = WarmStart(model, count)
    out = {}
    truth = None
    for name, mixed, guess, limit in forms:
        fam = Family(insts, mixed=mixed, guess_limit=limit, lockstep_block=lockstep_block)
        x = torch.empty(count, N_DOFS, dtype=torch.float64, device="cuda")
        _, rep = fam.batch.alloc()
        if guess == "exact":
            if truth is None:
                raise ValueError("the exact-coarse form needs a solved form before it")
            exact = torch.from_numpy(truth.astype(np.float32)).cuda()

        def run():
            if guess == "net":
                ws.guess(feats, x)
            elif guess == "exact":
                A.warmstart_prolong(ws.mesh, exact, COARSE, ws.mode, x)
            else:
                x.zero_()
            fam.solve(x, rep)

        run()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            run()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        R = A.Batch.reports(rep)
        if truth is None:
            truth = coarse_means(x.cpu().numpy())
        it = R["iters"].astype(np.float64)
        out[name] = {"seconds": float(np.median(ts)), "solves_per_s": count / float(np.median(ts)),
                     "iters_median": float(np.median(it)), "iters_p90": float(np.percentile(it, 90)),
                     "iters_mean": float(it.mean()), "rejected": int(R["guess_rejected"].sum()),
                     "converged": int((R["status"] == 0).sum()), "max_rel_res": float(R["rel_res"].max()),
                     "rel_res0_median": float(np.median(R["rel_res0"])), "iters": R["iters"].copy()}
        if log:
            o = out[name]
            log("%-24s %.3f s (%.1f solves/s)  iters median %.0f p90 %.0f  rejected %d  converged %d/%d  "
                "max rel-res %.2e  rel-res0 median %.3g" % (name, o["seconds"], o["solves_per_s"], o["iters_median"],
                                                            o["iters_p90"], o["rejected"], o["converged"], count,
                                                            o["max_rel_res"], o["rel_res0_median"]))
        del fam
        torch.cuda.empty_cache()
    le = np.array([math.log10(i.eps) for i in insts])
    out["by_log10_eps"] = []
    names = [f[0] for f in forms]
    for lo in range(-6, -1):
        sel = (le >= lo) & (le < lo + 1)
        if not sel.any():
            continue
        row = {"log10_eps": [lo, lo + 1], "count": int(sel.sum())}
        for name in names:
            row[name] = float(np.median(out[name]["iters"][sel]))
        out["by_log10_eps"].append(row)
        if log:
            log("  log10 eps in [%d,%d): %3d instances, median iterations %s" % (
                lo, lo + 1, row["count"], ", ".join("%s %.0f" % (n, row[n]) for n in names)))
    pred = ws.coarse(feats).cpu().numpy()
    err = np.linalg.norm(pred - truth, axis=1) / np.maximum(np.linalg.norm(truth, axis=1), 1e-300)
    out["coarse_rel_err"] = err
    out["coarse_rel_err_median"] = float(np.median(err))
    out["coarse_rel_err_p90"] = float(np.percentile(err, 90))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        ws.guess(feats, x)
    torch.cuda.synchronize()
    out["guess_ms"] = (time.perf_counter() - t0) / 20 * 1e3
    if log:
        log("coarse prediction rel. error median %.3f p90 %.3f (zero guess: 1); network + prolongation %.3f ms "
            "for %d instances" % (out["coarse_rel_err_median"], out["coarse_rel_err_p90"], out["guess_ms"], count))
    return out


def main(argv=None):
    import argparse
    import sys
    ap = argparse.ArgumentParser(description="Train and evaluate the learned initial guess.")
    ap.add_argument("--train-count", type=int, default=20000)
    ap.add_argument("--train-seed", type=int, default=1)
    ap.add_argument("--test-count", type=int, default=512)
    ap.add_argument("--test-seed", type=int, default=2)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--out", default=None, help="where to write the trained model (.npz)")
    ap.add_argument("--model", default=None, help="evaluate this model instead of training one")
    args = ap.parse_args(argv)

    def log(m):
        print(m, file=sys.stderr, flush=True)

    if args.model:
        model = load(args.model)
    else:
        X, Y, its = generate(args.train_count, args.train_seed, log=log)
        log("training solves: iterations median %.0f p90 %.0f" % (np.median(its), np.percentile(its, 90)))
        model = train(X, Y, epochs=args.epochs, log=log)
        if args.out:
            save(model, args.out)
            log("model written to %s" % args.out)
    evaluate(model, args.test_count, args.test_seed, log=log)


if __name__ == "__main__":
    main()
