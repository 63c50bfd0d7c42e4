"""CPU oracle for phaseless AFQMC -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 (complex128) implementation of the per-step, per-walker
path of phaseless AFQMC with a Hamiltonian in Cholesky form, written from
Motta & Zhang, "Ab initio computations of molecular systems by the
auxiliary-field quantum Monte Carlo method" (arXiv:1711.02242):

* ``afqmc``  -- setup, overlap / Green's function (Theorem 1), force bias
  (eq:fb, eq:precomputing2), Taylor propagation (Theorem 1.4, Sec. III.D.2),
  local energy (eq:localenergy2, eq:localenergy3), phaseless weight
  (eq:if_rle), modified Gram-Schmidt (Sec. III.D.5), comb population control
  (Sec. III.D.4), mixed estimator (eq:localenergy).
* ``fock``   -- brute-force second quantization on the full Fock sector of a
  tiny system (exact diagonalization), used to pin ``afqmc``.
* ``reblock``-- weighted reblocking error analysis (App. C).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding in ``paper_1711_02242_amd``) never imports, calls or links
anything here, and this package shares no code with it: the two meet only in
the seeded inputs of ``synthetic/``.
"""
