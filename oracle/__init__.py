"""CPU oracle for partitioned synchronous Jacobi.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import or run anything here.  The product
library (``paper_2112_02377_amd``) never imports, links or calls this package,
and this package never imports the product: the two share only the seeded
input generators, which hold none of the method's arithmetic.

* ``jacobi_ref.c``  plain C FP64 sweeps, solve, full-storage adjoint
  (built into ``libjacobi_ref.so`` by ``build.py``).
* ``partition.py``  band-row / sparsity-pattern / substructuring partitioner.
* ``ref.py``        ctypes wrappers and the derived references (batched,
  refinement target, conductivity gradient).

Parity status of every function is listed in ``ref.py``'s module docstring.
"""
