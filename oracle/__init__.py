"""Plain FP64 CPU oracle for the infinite binary MERA energy/gradient path and its Stiefel-manifold optimiser.

This package is TEST INFRASTRUCTURE. Only the test-suite, the smoke check of the package entry point and the
CPU-baseline leg of the benchmark may import it. The product library never calls it, and it shares no code
with the HIP path: it is written directly from Hauru, Van Damme & Haegeman, "Riemannian optimization of
isometric tensor networks" (arXiv:2007.03638), in numpy/scipy, at double precision.

Modules
  model     blocked 3-site Hamiltonian terms (Sec. 4 critical Ising, XXZ) and closed-form ground energies
  mera      binary-MERA layer maps, scale-invariant fixed point, energy, environments, Euclidean gradient (Sec. 4, App. B)
  manifold  Stiefel projection, polar retraction, projection transport, Hilbert-space preconditioner (Sec. 2, Sec. 3)
  optim     L-BFGS two-loop, Wolfe / approximate-Wolfe line search, optimisation driver (Sec. 3)
  finite    explicit state vector of a small finite binary MERA (brute-force pin of the layer maps)

Parity status: every function here is pinned by a test under tests/ (test_oracle_*.py) against closed forms,
invariants, brute force or finite differences, except the final optimiser trajectory values, which the paper
does not print ("parity unpinned" for the end energies of a full run; only invariants of the run are pinned).
"""
