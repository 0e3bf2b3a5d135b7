"""FP64 CPU oracle for complex constrained total-variation denoising (Gao & Cao,
arXiv 2109.05496) and its proximal-gradient phase-retrieval application.

This package is TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it. The product path (the
HIP library and its Python binding) never imports, calls or links anything here,
and nothing here imports the product path. The two share no code: the oracle
works in the paper's unpadded shapes ((m-1) x n and m x (n-1) difference arrays,
separate real and imaginary planes) in float64, the GPU path in padded complex64.

Modules
-------
tv        finite differences (Eqs. 5-6), the four complex TV seminorms (Eqs. 7-10),
          projections P_C (Eq. 26, plus a support mask) and P_S (Eqs. 20, 33, 35, 37),
          the FGP iteration (Algorithm 2 with Eqs. 18-19), the dual function
          (Eq. 16 / Appendix A) and the duality gap.
real_fgp  an independently written real-valued constrained FGP (the real-image
          special case that Section IV-B generalises); used only as a pin.
pdhg      dense-matrix primal-dual brute force for tiny images; used only as a pin.
adjoint   reverse-mode derivative of the K-step FGP map (b, lambda) -> x_K, written
          by hand, plus an independent float64 torch-autograd reference.
pr        angular-spectrum propagation (Eq. 23), the amplitude data term (Eq. 24)
          and its gradient (Eq. 27), and FISTA (Algorithm 1) with the FGP prox.

Parity status: every function is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py``. The phase-retrieval loop ``pr.fista`` is pinned by
Algorithm 1's closed form on a problem without measurements (every iterate a
known multiple of x_0) and by the qualitative behaviour on real data; the paper
prints no iterates of its own.
"""
