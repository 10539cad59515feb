"""Run one optimisation job through the library and print a JSON summary.

python -m paper_2007_03638_amd.run_config --chi 4 --T 2 --prec fp64 --iters 200 --seed 0 [--model tfim --param 1.0]
    [--polish 1e-5] [--grad-tol 1e-10] [--progress 10] [--save out.npz] [--init in.npz --iter-offset N]
    [--time-limit S] [--polish-iters K]

Initial tensors are Haar-random (seeded), or read from an .npz written by --save (a run continued in pieces: the
optimiser's history and warm starts start afresh at each piece; --iter-offset N counts the iterations already
done against --iters). The Hamiltonian is the blocked 3-site TFIM or XXZ term. With --progress N the run prints
every N-th iteration to stderr. --time-limit stops stepping after S seconds (the tensors are then saved as
usual). --polish-iters K then runs K iterations of the plain FP64 form from the final point (fresh history), the
polishing phase of a reduced-precision run that did not reach its polishing threshold, and reports the energy of
the final point in the run's precision and in FP64.
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
    ap.add_argument("--extrapolate", type=int, default=0,
                    help="Krylov warm starts extrapolated along the step (1), or from the last solution (-1); "
                         "0: library default (extrapolated)")
    ap.add_argument("--save", default="", help="write the final tensors to this .npz")
    ap.add_argument("--init", default="", help="initial tensors from an .npz written by --save")
    ap.add_argument("--iter-offset", type=int, default=0, help="iterations already done (with --init)")
    ap.add_argument("--time-limit", type=float, default=0.0, help="stop stepping after this many seconds")
    ap.add_argument("--krylov-tol", type=float, default=0.0, help="Krylov relative residual (0: default)")
    ap.add_argument("--precision-check", action="store_true",
                    help="report the energy of the final point in the run's precision and in FP64")
    ap.add_argument("--inter-limit-gib", type=float, default=0.0,
                    help="context intermediate limit in GiB (0: library default, 32)")
    ap.add_argument("--polish-iters", type=int, default=0,
                    help="FP64 iterations from the final point after the run (fresh history)")
    a = ap.parse_args()

    from . import api, inputs
    ctx = api.Context(0)
    if a.progress:
        ctx.set_verbose(1)
    if a.inter_limit_gib > 0:
        ctx.set_intermediate_limit(int(a.inter_limit_gib * (1 << 30)))
    ter = a.geometry == "ternary"
    d = 2 if ter else 4
    dims = api.layer_dims(a.T, a.chi, d, a.geometry)
    if a.init:
        z = np.load(a.init)
        init = [z[f"arr_{i}"] for i in range(2 * (a.T + 1))]
    else:
        init = [m for pair in inputs.mera_init(a.seed, dims, w_legs=3 if ter else 2) for m in pair]
    if ter:
        h3 = api.h2_tfim(a.param) if a.model == "tfim" else api.h2_xxz(a.param)
    else:
        h3 = api.h3_tfim(a.param) if a.model == "tfim" else api.h3_xxz(a.param)
    t0 = time.perf_counter()
    opt = ctx.optimizer(T=a.T, chi=a.chi, h3=h3, init=init, prec=a.prec, m=a.m, max_iter=a.iters - a.iter_offset,
                        grad_tol=a.grad_tol, polish_tol=a.polish, method=a.method, retraction=a.retraction,
                        grassmann_w=a.grassmann_w, ev_gamma=a.ev_gamma, d=d, geometry=a.geometry,
                        krylov={"extrapolate": a.extrapolate, "tol": a.krylov_tol})
    done, st = False, None
    history = []
    stopped = ""
    while not done:
        done, st = opt.step()
        it = st["iterations"] + a.iter_offset
        history.append((it, st["evaluations"], st["energy"], st["gnorm"], st["polish_iter"]))
        if a.progress and (it % a.progress == 0 or done):
            print(f"[run] iter {it} evals {st['evaluations']} e {st['energy']:.12f} "
                  f"|G| {st['gnorm']:.3e} t {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        if not done and a.time_limit > 0 and time.perf_counter() - t0 > a.time_limit:
            stopped = "time limit"
            break
    dt = time.perf_counter() - t0
    final = opt.final()
    if a.save:
        np.savez(a.save, *final)
    polish = None
    check = None
    if a.precision_check:
        u, w = final[0::2], final[1::2]
        e_run = ctx.energy_grad(a.T, a.chi, u, w, h3, prec=a.prec, d=d, geometry=a.geometry)["energy"]
        e_64 = ctx.energy_grad(a.T, a.chi, u, w, h3, prec="fp64", d=d, geometry=a.geometry)["energy"]
        check = dict(energy_run_precision=e_run, energy_fp64=e_64, rel_diff=abs(e_run - e_64) / abs(e_64))
    if a.polish_iters > 0:
        u, w = final[0::2], final[1::2]
        e_run = ctx.energy_grad(a.T, a.chi, u, w, h3, prec=a.prec, d=d, geometry=a.geometry)["energy"]
        e_64 = ctx.energy_grad(a.T, a.chi, u, w, h3, prec="fp64", d=d, geometry=a.geometry)["energy"]
        t1 = time.perf_counter()
        pol = ctx.optimizer(T=a.T, chi=a.chi, h3=h3, init=final, prec="fp64", m=a.m, max_iter=a.polish_iters,
                            grad_tol=a.grad_tol, polish_tol=0.0, method=a.method, retraction=a.retraction,
                            grassmann_w=a.grassmann_w, ev_gamma=a.ev_gamma, d=d, geometry=a.geometry)
        pdone, pst = False, None
        while not pdone:
            pdone, pst = pol.step()
            if a.progress:
                print(f"[polish] iter {pst['iterations']} evals {pst['evaluations']} e {pst['energy']:.15f} "
                      f"|G| {pst['gnorm']:.3e} t {time.perf_counter() - t1:.1f} s", file=sys.stderr, flush=True)
        pfinal = pol.final()
        if a.save:
            np.savez(a.save.replace(".npz", "_polished.npz"), *pfinal)
        polish = dict(energy_run_precision_at_final=e_run, energy_fp64_at_final=e_64,
                      rel_diff=abs(e_run - e_64) / abs(e_64), iterations=pst["iterations"],
                      evaluations=pst["evaluations"], energy=pst["energy"], gnorm=pst["gnorm"],
                      status=pst["status"], seconds=time.perf_counter() - t1)
    out = dict(chi=a.chi, T=a.T, prec=a.prec, method=a.method, retraction=a.retraction, grassmann_w=a.grassmann_w,
               seed=a.seed, model=a.model, param=a.param,
               geometry=a.geometry, energy=st["energy"], energy_per_spin=st["energy"] / (1 if ter else 2),
               gnorm=st["gnorm"],
               iterations=st["iterations"] + a.iter_offset, evaluations=st["evaluations"], status=st["status"],
               stopped=stopped, init=a.init, polish=polish, precision_check=check,
               polish_iter=st["polish_iter"], seconds=dt, tflops=2 * st["macs"] / dt / 1e12,
               krylov_applications=st["krylov_applications"],
               krylov_per_eval=st["krylov_applications"] / max(1, st["evaluations"]),
               history=history[:: max(1, len(history) // 50)])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
