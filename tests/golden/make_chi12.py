"""Writes tests/golden/eval_chi12_T2.npz and eval_chi12_T2_near.npz: the oracle's energy, Euclidean gradient and
preconditioner density matrices of binary-MERA evaluations at chi = 12, T = 2 (TFIM h = 1, d = 4), at Haar tensors
from seed 12 (energy near zero) and at tensors near the identity from seed 13 (inputs.mera_init_near_identity,
eps = 0.1: energy far from zero, so that relative energy errors are meaningful).

At chi = 12 the GPU evaluation takes the kernel paths of the benchmark's bond dimension (chi^3 = 1728 and
chi^4 = 20736 are multiples of the 192-wide tiles, and the K = chi^4 environment reductions run split-K), while the
oracle needs minutes; the values are stored once. Calls only oracle/ and the seeded input generators.

Usage: python tests/golden/make_chi12.py [haar|near]   (both when no argument is given)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import mera, model  # noqa: E402
from paper_2007_03638_amd import inputs  # noqa: E402

CHI, T = 12, 2
CASES = {"haar": (12, 0.0, "eval_chi12_T2.npz"), "near": (13, 0.1, "eval_chi12_T2_near.npz")}


def make(kind):
    seed, eps, name = CASES[kind]
    out_path = os.path.join(HERE, name)
    t0 = time.time()
    dims = mera.layer_dims(CHI, T)
    params = inputs.mera_init(seed, dims) if eps == 0.0 else inputs.mera_init_near_identity(seed, dims, eps)
    h3 = model.tfim_h3(1.0)
    ref = mera.evaluate(params, h3, CHI, T)
    rdms = mera.preconditioner_rdms(ref["rhos"], params, dims)
    e_bottom = mera.energy_bottom(params, h3, CHI, T)
    out = dict(chi=CHI, T=T, seed=seed, eps=eps, energy=ref["energy"], energy_bottom=e_bottom)
    for t in range(T + 1):
        out[f"Du{t}"], out[f"Dw{t}"] = ref["grads"][t]
        out[f"rho_u{t}"], out[f"rho_w{t}"] = rdms[t]
    np.savez_compressed(out_path, **out)
    print(f"{kind}: energy {ref['energy']!r} (via full descent {e_bottom!r}); {time.time() - t0:.0f} s -> {out_path}")


if __name__ == "__main__":
    for k in (sys.argv[1:] or list(CASES)):
        make(k)
