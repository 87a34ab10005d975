"""CPU oracle for the fixed-budget Gaussian volume encoder.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, float64 NumPy
statement of what the encoder computes.  It exists so that the HIP path can be
checked against something written independently from the paper:

* ``oracle.field``  -- truncated / untruncated evaluation of the weighted
  anisotropic Gaussian sum, the sum-of-squares loss, its analytic gradient,
  Adam and the refinement loop (Sec. III-C eq:field as read for an
  unnormalised weighted sum; Sec. III-F; Sec. III-G).
* ``oracle.alloc``  -- the structure-aware fixed-budget allocation
  (Sec. III-E, Table "Implemented pipeline stages" rows S1a-S1e).
* ``oracle.mlp``    -- the warm-start MLP reference (not in the paper; defined
  by its shapes only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the C-ABI library and
its Python binding) never imports, links or executes anything here, and this
package never imports the product path.
"""
