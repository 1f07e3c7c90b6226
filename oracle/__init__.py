"""CPU oracle for the low-rank isogeometric Tucker solver (TEST INFRASTRUCTURE).

This package is a plain, slow, FP64 numpy/scipy implementation of what the
paper "A low-rank isogeometric solver based on Tucker tensors" (Montardini,
Sangalli, Tani) computes.  It exists only to check the GPU library:

* only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
  ``bench.py`` may import it;
* it shares no code with the GPU path (``paper_2306_00632_amd``) and never
  imports it; the two meet only in ``workloads`` (seeded recipes, no method
  arithmetic);
* every function cites the passage of the paper it follows.

Modules
-------
bspline   Sec. 2.1 (Cox-de Boor), App. A (1D weighted matrices, load vectors)
tucker    Sec. 2.3 (mode products, Tucker format, eq. tt_product, dot, sum),
          Sec. 4.1 (Algorithm 1 relative truncation, Algorithm 2 dynamic)
expsum    Sec. 4.2 Proposition 1 (exponential sums for 1/x) via Remez
fd        Sec. 4.2 (Algorithm 3 exact FD, Algorithm 4 low-rank FD), App. B
tpcg      Sec. 4.3 Algorithm 5 (TPCG)
fullpcg   full-tensor PCG with exact FD (reference solutions)
problem   builds operator / rhs objects from ``workloads`` recipes
"""
