"""Train the learned refinement preconditioner on synthetic 3D diffusion matrices and
evaluate it on held-out 64^3 systems.

Training set: matrices from ``workloads.diffusion3d_7pt`` with grid edges uniform on
[edge_lo, edge_hi], lognormal coefficient spread sigma ~ U(sigma_lo, sigma_hi) and the
anisotropy factor of the calibrated 64^3 law (workloads/c2_law.json), one seed per
matrix.  Each epoch streams the same matrices (regenerated from their seeds on host
threads while the GPU trains, never stored): their (r, e) pairs come from plain DD
Jacobi-CG iterates toward a random DD solution, and ``steps_per_matrix`` Adam steps
are taken on them; the learning rate decays geometrically over all epochs.  Every
arithmetic step runs in the HIP library (network forward/backward/Adam, CG, SpMV).

Evaluation: the two 64^3 systems of the solver benchmark and held-out 64^3 systems
(fresh seeds, the training sigma law, the same anisotropy), each solved to a relative
residual of 1e-28 by plain DD Jacobi-CG, Jacobi refinement and learned refinement
(binary64 and binary32 inner solves); the network's forward pass is timed separately
and included in the learned solve time.

Usage:  python -m paper_2412_17510_amd.train_mpnn --matrices 2000 --epochs 4 --out <ckpt.npz>
        python -m paper_2412_17510_amd.train_mpnn --eval-only --ckpt <ckpt.npz> --eval 200
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
DEFAULT_CKPT = os.path.join(HERE, "data", "mpnn_diffusion.npz")


def _log(*a):
    print("[train_mpnn]", *a, flush=True)


def _workloads():
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import workloads
    return workloads


def _law_az():
    wl = _workloads()
    from workloads.condition import load_law
    return load_law()["systems"][0]["az"]


def train(n_matrices=2000, steps_per_matrix=2, edge_lo=24, edge_hi=48, sigma_lo=1.5, sigma_hi=3.0, seed=0,
          lr=3e-3, lr_final=3e-4, log_every=250, epochs=1, az=None):
    """Returns (theta, history, curve).  history: list of (epoch, matrix index, n, mean
    loss of its pairs before its first step); curve: mean of those losses per epoch."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    from . import _binding as mp
    from . import learned
    wl = _workloads()
    if az is None:
        az = _law_az()
    rng = np.random.default_rng([seed, 1])
    law = [(int(rng.integers(edge_lo, edge_hi + 1)), float(rng.uniform(sigma_lo, sigma_hi)),
            int(rng.integers(1, 2 ** 31 - 1))) for _ in range(n_matrices)]

    def make(item):
        m, sg, ms = item
        rp, ci, a = wl.diffusion3d_7pt(m=m, sigma=sg, az=az, seed=ms)
        return rp, ci, a, wl.random_mp(rp.size - 1, 2, np.random.default_rng(ms))

    net = mp.Mpnn()
    net.set_params(learned.init_params(seed))
    step = 0
    total_steps = epochs * n_matrices * steps_per_matrix
    history, curve = [], []
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=4) as pool:
        for ep in range(epochs):
            pending = [pool.submit(make, law[i]) for i in range(min(8, n_matrices))]
            ep_loss, run_loss, run_cnt = 0.0, 0.0, 0
            for i in range(n_matrices):
                rp, ci, a, xt_h = pending.pop(0).result()
                if i + len(pending) + 1 < n_matrices:
                    pending.append(pool.submit(make, law[i + len(pending) + 1]))
                n = rp.size - 1
                A = mp.Csr.from_numpy(rp, ci)
                ad = torch.from_numpy(a).cuda()
                xt = torch.from_numpy(xt_h).cuda()
                # the pairs' DD CG runs under a tile plan (rows summed sequentially) rather than
                # the plan-free one-row-per-wavefront kernel
                R, E = learned.cg_pairs(A, ad, xt, plan=mp.mp_plan_create(A, 2, False, 2, 6, 512))
                g = mp.Graph(A, ad)
                for s in range(steps_per_matrix):
                    frac = step / max(1, total_steps - 1)
                    lr_s = lr * (lr_final / lr) ** frac
                    net.zero_grads()
                    losses = mp.mp_mpnn_loss_grad(net, g, R, E)
                    if s == 0:
                        lm = float(losses.mean())
                        history.append((ep, i, n, lm))
                        ep_loss += lm
                        run_loss += lm
                        run_cnt += 1
                    step += 1
                    net.adam_step(step, lr=lr_s, grad_scale=1.0 / losses.size)
                g.destroy()
                del A, ad, xt, R, E
                if (i + 1) % log_every == 0 or i + 1 == n_matrices:
                    torch.cuda.synchronize()
                    _log("epoch %d matrix %d/%d  mean loss (last %d) %.5f  %.1f s" % (
                        ep + 1, i + 1, n_matrices, run_cnt, run_loss / max(1, run_cnt), time.perf_counter() - t0))
                    run_loss, run_cnt = 0.0, 0
            curve.append(ep_loss / n_matrices)
            _log("epoch %d mean pair loss %.5f" % (ep + 1, curve[-1]))
    return net.get_params(), history, curve


def _solve(fn, *args, **kw):
    return fn(*args, **kw)


def evaluate(theta, n_systems=8, m=64, sigma_lo=1.5, sigma_hi=3.0, seed=7, inner=("fp64", "fp32"),
             include_bench=True, log=True, az=None):
    """Per-system and summary results of plain DD CG, Jacobi refinement and learned
    refinement on held-out m^3 systems (relative residual 1e-28)."""
    import torch
    from . import _binding as mp
    wl = _workloads()
    if az is None:
        az = _law_az()
    net = mp.Mpnn()
    net.set_params(theta)
    rng = np.random.default_rng([seed, 2])
    systems = []
    if include_bench:
        from workloads.condition import load_law
        for law in load_law()["systems"]:   # the 64^3 systems of the solver benchmark
            systems.append((law["sigma"], law["seed"]))
    while len(systems) < n_systems:
        systems.append((float(rng.uniform(sigma_lo, sigma_hi)), int(rng.integers(10 ** 6, 2 ** 31 - 1))))
    inner_rtol = {"fp64": 1e-8, "fp32": 1e-5}
    rows = []
    for k, (sg, ms) in enumerate(systems):
        rp, ci, a = wl.diffusion3d_7pt(m=m, sigma=sg, az=az, seed=ms)
        n = rp.size - 1
        A = mp.Csr.from_numpy(rp, ci)
        ad = torch.from_numpy(a).cuda()
        bd = torch.from_numpy(wl.random_mp(n, 2, np.random.default_rng(ms))).cuda()
        ytmp = torch.empty((2, n), dtype=torch.float64, device="cuda")
        plan, _ = mp.mp_plan_autotune(A, 2, ad, bd, ytmp, reps=3)
        # learned M (forward pass timed: graph set-up + network)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = mp.Graph(A, ad)
        M = mp.mp_mpnn_forward(net, g)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        g.destroy()
        rec = {"sigma": round(sg, 4), "seed": ms, "n": n, "forward_s": round(t_fwd, 5)}
        x = torch.zeros((2, n), dtype=torch.float64, device="cuda")
        info = mp.mpkrylov_cg(A, ad, bd, x, plan=plan, rtol=1e-28, max_iter=200000)
        rec["plain_dd_cg"] = {"s": round(info["seconds"], 5), "iters": info["iters"], "status": info["status"],
                              "relres": info["relres"]}
        for inn in inner:
            for name, fn, extra in (("ir_%s_jacobi" % inn, mp.mpkrylov_ir, {}),
                                    ("ir_%s_learned" % inn, mp.mpkrylov_ir_learned, {"m_values": M})):
                x.zero_()
                kw = dict(plan=plan, rtol=1e-28, inner=inn, inner_rtol=inner_rtol[inn], inner_max_iter=50000,
                          max_outer=60, max_iter=200000)
                if "m_values" in extra:
                    info = fn(A, ad, extra["m_values"], bd, x, **kw)
                else:
                    info = fn(A, ad, bd, x, **kw)
                secs = info["seconds"] + (t_fwd if "m_values" in extra else 0.0)
                rec[name] = {"s": round(secs, 5), "iters": info["iters"], "outer": info["outer_iters"],
                             "status": info["status"], "fell_back": info["fell_back"], "relres": info["relres"]}
        rows.append(rec)
        if log:
            _log("eval %d/%d sigma %.2f: cg %d it %.3f s | ir64 jac %d it %.3f s | ir64 learned %d it %.3f s"
                 % (k + 1, len(systems), sg, rec["plain_dd_cg"]["iters"], rec["plain_dd_cg"]["s"],
                    rec["ir_fp64_jacobi"]["iters"], rec["ir_fp64_jacobi"]["s"], rec["ir_fp64_learned"]["iters"],
                    rec["ir_fp64_learned"]["s"]))
        del A, ad, bd, x, M, plan
        torch.cuda.empty_cache()
    return {"systems": rows, "summary": summarize(rows)}


def summarize(rows):
    keys = [k for k in rows[0] if isinstance(rows[0][k], dict)]
    out = {"n_systems": len(rows)}
    for k in keys:
        secs = np.array([r[k]["s"] for r in rows])
        its = np.array([r[k]["iters"] for r in rows])
        ok = sum(1 for r in rows if r[k]["status"] == 0)
        out[k] = {"solves_per_s": round(float(len(rows) / secs.sum()), 3), "mean_s": round(float(secs.mean()), 5),
                  "mean_iters": round(float(its.mean()), 1), "converged": ok,
                  "max_relres": float(max(r[k]["relres"] for r in rows))}
        fb = [r[k].get("fell_back", 0) for r in rows]
        out[k]["fell_back"] = int(sum(fb))
    base = out.get("plain_dd_cg", {}).get("mean_s")
    for k in keys:
        if base:
            out[k]["speedup_vs_plain_dd_cg"] = round(base / out[k]["mean_s"], 3)
    for inn in ("fp64", "fp32"):
        j, l_ = out.get("ir_%s_jacobi" % inn), out.get("ir_%s_learned" % inn)
        if j and l_:
            out["learned_vs_jacobi_inner_iters_%s" % inn] = round(l_["mean_iters"] / j["mean_iters"], 4)
    return out


def main():
    _workloads()
    from workloads import configs
    c4 = configs.load("c4")
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--matrices", type=int, default=c4["train_matrices"])
    ap.add_argument("--steps-per-matrix", type=int, default=2)
    ap.add_argument("--epochs", type=int, default=1)
    ap.add_argument("--seed", type=int, default=c4["train_seed"])
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--out", default=DEFAULT_CKPT)
    ap.add_argument("--eval", type=int, default=0, help="held-out 64^3 systems to evaluate after training")
    ap.add_argument("--eval-out", default=None)
    ap.add_argument("--eval-only", action="store_true")
    ap.add_argument("--ckpt", default=DEFAULT_CKPT)
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    from . import learned
    if args.eval_only:
        theta = learned.load(args.ckpt)
    else:
        t0 = time.perf_counter()
        theta, hist, curve = train(args.matrices, args.steps_per_matrix, edge_lo=c4["train_edge_lo"],
                                   edge_hi=c4["train_edge_hi"], sigma_lo=c4["train_sigma_lo"],
                                   sigma_hi=c4["train_sigma_hi"], seed=args.seed, lr=args.lr, epochs=args.epochs)
        secs = time.perf_counter() - t0
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        first = float(np.mean([h[3] for h in hist[:50]]))
        last = float(np.mean([h[3] for h in hist[-50:]]))
        learned.save(args.out, theta, matrices=args.matrices, steps_per_matrix=args.steps_per_matrix,
                     epochs=args.epochs, seed=args.seed, train_seconds=secs, loss_first50=first, loss_last50=last,
                     az=_law_az(), epoch_loss=np.asarray(curve))
        _log("saved %s: %d matrices x %d epochs in %.1f s, mean pair loss %.4f (first 50) -> %.4f (last 50); "
             "per epoch %s" % (args.out, args.matrices, args.epochs, secs, first, last,
                               " ".join("%.4f" % c for c in curve)))
    if args.eval > 0:
        res = evaluate(theta, n_systems=args.eval, m=c4["eval_m"], sigma_lo=c4["eval_sigma_lo"],
                       sigma_hi=c4["eval_sigma_hi"], seed=c4["eval_seed"])
        _log(json.dumps(res["summary"]))
        if args.eval_out:
            with open(args.eval_out, "w") as f:
                json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
