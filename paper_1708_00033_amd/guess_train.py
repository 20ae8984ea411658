"""Train the learned initial guess on converged densities from this SCF and
evaluate it against the SAD start.

    python -m paper_1708_00033_amd.guess_train --train 2000 --eval 0 \\
        --out paper_1708_00033_amd/models/guess_water.npy --report guess_report.json
    python -m paper_1708_00033_amd.guess_train --eval-only paper_1708_00033_amd/models/guess_water.npy \\
        --eval 8 --report guess_eval.json

Data: seeded water clusters of 4-32 molecules (training) and of 128
molecules (evaluation).  The training clusters' FP64 SCFs from SAD run as
batches (hfx_batch_scf); then for each cluster the library writes the pair
features and the converged-minus-SAD blocks in the pair frames
(hfx_guess_setup / hfx_guess_targets_dev).  Training runs
the library's BF16 MFMA forward/backward and Adam (hfx_guess_grad_dev,
hfx_guess_adam) on minibatches gathered on the device.  Evaluation: SCF
iterations, SCF time and the converged energy from SAD and from the network.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np


def log(*a):
    print("[guess]", *a, flush=True)


def collect(mols, hfx, torch, stream, chunk=128):
    """Per pair type: features (rows) and target blocks, from converged SCF.
    The SCFs run as batches of `chunk` molecules of similar size
    (hfx_batch_scf, iterations replayed from HIP graphs); the features and
    targets of each molecule then come from a single-molecule context."""
    X = [[], [], []]
    T = [[], [], []]
    bctx = hfx.Context(device=0)
    ctx = hfx.Context(device=0)
    iters = []
    t0 = time.time()
    order = sorted(range(len(mols)), key=lambda i: mols[i].nbf)
    done = 0
    for b0 in range(0, len(order), chunk):
        part = [mols[i] for i in order[b0:b0 + chunk]]
        bctx.load_batch(part)
        res, Drag = bctx.batch_scf(graph=1)
        nbf, _, off, _ = bctx.layout
        for j, m in enumerate(part):
            if not res[j]["converged"]:
                log(f"a cluster of {m.natom // 3} waters did not converge; skipped")
                continue
            iters.append(res[j]["iterations"])
            n = int(nbf[j])
            D = Drag[int(off[j]):int(off[j]) + n * n].reshape(n, n)
            ctx.load(m)
            Dsad = ctx.sad_density()
            counts = ctx.guess_setup()
            Xh, _, _ = ctx.guess_features()
            dD = torch.tensor(D, device="cuda")
            dS = torch.tensor(Dsad, device="cuda")
            dT = torch.empty(ctx.guess_packed_size(), dtype=torch.float32, device="cuda")
            ctx.guess_targets_dev(dD.data_ptr(), dS.data_ptr(), dT.data_ptr(), stream.cuda_stream)
            stream.synchronize()
            Th = dT.cpu().numpy()
            ro, to = 0, 0
            for t, (c, w) in enumerate(zip(counts, hfx.GUESS_HEAD_OUT)):
                X[t].append(Xh[ro:ro + c])
                T[t].append(Th[to:to + c * w].reshape(c, w))
                ro += c
                to += c * w
        done += len(part)
        log(f"collected {done}/{len(mols)} clusters ({time.time() - t0:.0f} s, "
            f"mean SAD-start iterations {np.mean(iters):.1f})")
    ctx.close()
    bctx.close()
    X = [np.concatenate(x) if x else np.zeros((0, hfx.GUESS_NFEAT), np.float32) for x in X]
    T = [np.concatenate(x) if x else np.zeros((0, w), np.float32) for x, w in zip(T, hfx.GUESS_HEAD_OUT)]
    return X, T, iters


def packed(Xd, Td, idx):
    X = __import__("torch").cat([Xd[t][idx[t]] for t in range(3)])
    T = __import__("torch").cat([Td[t][idx[t]].reshape(-1) for t in range(3)])
    return X.contiguous(), T.contiguous(), [int(len(i)) for i in idx]


def evaluate(net, mols, hfx, tag):
    out = []
    ctx = hfx.Context(device=0)
    for j, m in enumerate(mols):
        ctx.load(m)
        r0 = ctx.scf()
        r1 = ctx.scf(model=net)
        import torch
        Dsad = ctx.sad_density()
        dD = torch.tensor(Dsad, device="cuda")
        ctx.guess_apply(net, dD.data_ptr(), 0)
        torch.cuda.synchronize()
        err_sad = float(np.linalg.norm(Dsad - r0["D"]))
        err_nn = float(np.linalg.norm(dD.cpu().numpy() - r0["D"]))
        row = dict(waters=m.natom // 3, nbf=ctx.nbf, sad_iterations=r0["iterations"],
                   start_density_error_sad=err_sad, start_density_error_learned=err_nn,
                   learned_iterations=r1["iterations"], sad_time_s=r0["t_total_s"], learned_time_s=r1["t_total_s"],
                   energy_sad=r0["energy"], energy_learned=r1["energy"],
                   dE=r1["energy"] - r0["energy"], guess_used=r1["guess_used"],
                   converged=bool(r0["converged"] and r1["converged"]))
        out.append(row)
        log(f"{tag} {j}: {row['waters']} waters, SAD {row['sad_iterations']} it {row['sad_time_s']:.2f} s, "
            f"learned {row['learned_iterations']} it {row['learned_time_s']:.2f} s, dE {row['dE']:.2e}, "
            f"guess_used {row['guess_used']}, |D0 - D| SAD {err_sad:.3f} learned {err_nn:.3f}")
    ctx.close()
    return out


def _means(ev):
    return dict(start_density_error_sad=float(np.mean([r["start_density_error_sad"] for r in ev])),
                start_density_error_learned=float(np.mean([r["start_density_error_learned"] for r in ev])),
                sad_iterations=float(np.mean([r["sad_iterations"] for r in ev])),
                learned_iterations=float(np.mean([r["learned_iterations"] for r in ev])),
                sad_time_s=float(np.mean([r["sad_time_s"] for r in ev])),
                learned_time_s=float(np.mean([r["learned_time_s"] for r in ev])),
                max_abs_dE=float(max(abs(r["dE"]) for r in ev))) if ev else None


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=2000, help="training clusters (4-32 waters)")
    ap.add_argument("--eval", type=int, default=8, help="128-water evaluation clusters")
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default="paper_1708_00033_amd/models/guess_water.npy")
    ap.add_argument("--report", default="")
    ap.add_argument("--eval-only", default="", help="evaluate this saved model, no training")
    a = ap.parse_args(argv)

    import torch
    import workloads as W
    from paper_1708_00033_amd import hfx

    if a.eval_only:
        net = hfx.GuessNet(0, np.load(a.eval_only))
        ev32 = evaluate(net, [W.water_cluster(32, 29_999)], hfx, "held-out 32")
        ev = evaluate(net, W.guess_eval_set(a.eval), hfx, "eval 128")
        rep = dict(model=a.eval_only, heldout32=ev32, eval128=ev, eval128_mean=_means(ev))
        if a.report:
            with open(a.report, "w") as fh:
                json.dump(rep, fh, indent=1)
        print(json.dumps(rep["eval128_mean"]), flush=True)
        return 0

    stream = torch.cuda.Stream()
    t0 = time.time()
    mols = W.guess_training_set(a.train)
    nval = max(1, a.train // 20)
    X, T, iters = collect(mols[:-nval], hfx, torch, stream)
    Xv, Tv, _ = collect(mols[-nval:], hfx, torch, stream)
    t_data = time.time() - t0
    rows = [len(x) for x in X]
    log(f"dataset: {sum(rows)} pairs {rows} from {len(iters)} clusters in {t_data:.0f} s")

    allX = np.concatenate(X).astype(np.float64)
    fmean = allX.mean(0)
    fscale = allX.std(0)
    fscale[fscale < 1e-3] = 1.0
    tscale = np.array([max(float(np.sqrt(np.mean(np.square(t.astype(np.float64))))), 1e-6) for t in T])
    net = hfx.GuessNet(0, hfx.GuessNet.init_params(a.seed, fmean, fscale, tscale))

    dev = torch.device("cuda")
    Xd = [torch.tensor(x, device=dev) for x in X]
    Td = [torch.tensor(t, device=dev) for t in T]
    Xvd = [torch.tensor(x, device=dev) for x in Xv]
    Tvd = [torch.tensor(t, device=dev) for t in Tv]
    Xval, Tval, cval = packed(Xvd, Tvd, [torch.arange(len(x), device=dev) for x in Xv])
    ntot = sum(rows)
    steps_per_epoch = max(1, math.ceil(ntot / a.batch))
    nsteps = a.epochs * steps_per_epoch
    g = torch.Generator(device="cpu").manual_seed(a.seed)
    s = stream.cuda_stream
    hist = []
    best = (float("inf"), None, -1)
    t1 = time.time()
    with torch.cuda.stream(stream):
        for step in range(nsteps):
            lr = 1e-5 + 0.5 * (a.lr - 1e-5) * (1 + math.cos(math.pi * step / nsteps))
            idx = [torch.randint(0, max(r, 1), (max(1, round(a.batch * r / ntot)),), generator=g).to(dev)
                   if r else torch.zeros(0, dtype=torch.long, device=dev) for r in rows]
            xb, tb, cb = packed(Xd, Td, idx)
            want = (step % steps_per_epoch == 0) or step == nsteps - 1
            loss = net.grad_dev(xb.data_ptr(), cb, tb.data_ptr(), s, want_loss=want)
            net.adam(lr, s)
            if want:
                vloss = net.grad_dev(Xval.data_ptr(), cval, Tval.data_ptr(), s)
                hist.append(dict(step=step, train_loss=loss, val_loss=vloss, lr=lr))
                log(f"epoch {step // steps_per_epoch}: train {loss:.4e} val {vloss:.4e} lr {lr:.2e}")
                if vloss < best[0]:
                    best = (vloss, net.get_params(), step)
        stream.synchronize()
    t_train = time.time() - t1
    net.set_params(best[1])     # the parameters with the lowest validation loss
    log(f"kept the parameters of step {best[2]} (validation loss {best[0]:.4e})")
    params = net.get_params()
    np.save(a.out, params)
    log(f"trained {nsteps} steps in {t_train:.1f} s; saved {a.out}")

    ev32 = evaluate(net, [W.water_cluster(32, 29_999)], hfx, "held-out 32")
    ev = evaluate(net, W.guess_eval_set(a.eval), hfx, "eval 128") if a.eval else []
    rep = dict(train_clusters=len(iters), val_clusters=nval, pairs=rows, data_s=t_data, train_s=t_train,
               steps=nsteps, batch=a.batch, epochs=a.epochs, history=hist, heldout32=ev32, eval128=ev,
               sad_start_iterations_train_mean=float(np.mean(iters)) if iters else None)
    rep["best_val_loss"] = best[0]
    rep["best_step"] = best[2]
    if ev:
        rep["eval128_mean"] = _means(ev)
    if a.report:
        with open(a.report, "w") as fh:
            json.dump(rep, fh, indent=1)
    print(json.dumps({k: rep[k] for k in ("train_clusters", "pairs", "data_s", "train_s", "steps")} |
                     {"eval128_mean": rep.get("eval128_mean"), "heldout32": ev32}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
