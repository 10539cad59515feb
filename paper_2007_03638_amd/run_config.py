"""Run one optimisation job through the library and print a JSON summary.

python -m paper_2007_03638_amd.run_config --chi 4 --T 2 --prec fp64 --iters 200 --seed 0 [--model tfim --param 1.0]
    [--polish 1e-5] [--grad-tol 1e-10] [--progress 10]

Initial tensors are Haar-random (seeded); the Hamiltonian is the blocked 3-site TFIM or XXZ term. With
--progress N the run proceeds through the step-wise API and prints every N-th iteration to stderr.
"""
import argparse
import json
import sys
import time

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--chi", type=int, default=4)
    ap.add_argument("--T", type=int, default=2)
    ap.add_argument("--prec", default="fp64")
    ap.add_argument("--iters", type=int, default=200)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--model", default="tfim", choices=["tfim", "xxz"])
    ap.add_argument("--geometry", default="binary", choices=["binary", "ternary"],
                    help="binary: three-site terms on blocked spins (d = 4); ternary: two-site terms on spins (d = 2)")
    ap.add_argument("--param", type=float, default=1.0)
    ap.add_argument("--polish", type=float, default=0.0)
    ap.add_argument("--grad-tol", type=float, default=1e-10)
    ap.add_argument("--m", type=int, default=8)
    ap.add_argument("--method", default="lbfgs", choices=["lbfgs", "cg", "ev"])
    ap.add_argument("--ev-gamma", type=float, default=20.0, help="Evenbly-Vidal shift (method ev)")
    ap.add_argument("--retraction", default="polar", choices=["polar", "exp"])
    ap.add_argument("--grassmann-w", action="store_true")
    ap.add_argument("--progress", type=int, default=0)
    ap.add_argument("--save", default="", help="write the final tensors to this .npz")
    a = ap.parse_args()

    from . import api, inputs
    ctx = api.Context(0)
    ter = a.geometry == "ternary"
    d = 2 if ter else 4
    dims = api.layer_dims(a.T, a.chi, d, a.geometry)
    init = [m for pair in inputs.mera_init(a.seed, dims, w_legs=3 if ter else 2) for m in pair]
    if ter:
        h3 = api.h2_tfim(a.param) if a.model == "tfim" else api.h2_xxz(a.param)
    else:
        h3 = api.h3_tfim(a.param) if a.model == "tfim" else api.h3_xxz(a.param)
    t0 = time.perf_counter()
    opt = ctx.optimizer(T=a.T, chi=a.chi, h3=h3, init=init, prec=a.prec, m=a.m, max_iter=a.iters,
                        grad_tol=a.grad_tol, polish_tol=a.polish, method=a.method, retraction=a.retraction,
                        grassmann_w=a.grassmann_w, ev_gamma=a.ev_gamma, d=d, geometry=a.geometry)
    done, st = False, None
    history = []
    while not done:
        done, st = opt.step()
        history.append((st["iterations"], st["evaluations"], st["energy"], st["gnorm"]))
        if a.progress and (st["iterations"] % a.progress == 0 or done):
            print(f"[run] iter {st['iterations']} evals {st['evaluations']} e {st['energy']:.12f} "
                  f"|G| {st['gnorm']:.3e} t {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    dt = time.perf_counter() - t0
    final = opt.final()
    if a.save:
        np.savez(a.save, *final)
    out = dict(chi=a.chi, T=a.T, prec=a.prec, method=a.method, retraction=a.retraction, grassmann_w=a.grassmann_w,
               seed=a.seed, model=a.model, param=a.param,
               geometry=a.geometry, energy=st["energy"], energy_per_spin=st["energy"] / (1 if ter else 2),
               gnorm=st["gnorm"],
               iterations=st["iterations"], evaluations=st["evaluations"], status=st["status"],
               polish_iter=st["polish_iter"], seconds=dt, tflops=2 * st["macs"] / dt / 1e12,
               krylov_applications=st["krylov_applications"],
               history=history[:: max(1, len(history) // 50)])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
